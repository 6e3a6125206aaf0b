"""The 30M-particle, order-10 cube (height 9: 13.97M non-empty leaves,
2.6e9 far pairs) in the compressed mixed mode on one GPU.

Its FP64 path needs about 284 GB (FP64 multipoles and local expansions of
16.4M cells), so the mixed modes store the leaf multipoles in FP32 only;
the plan then needs about 240 GB.  The reference is the exact direct sum at
seeded targets over all 3e7 sources (the oracle, on the host); the bound
is the FP64 FMM's own error at this density and order, measured on the
twin, plus the mixed mode's gate margin.
Parity with the oracle FMM at the same density and order is the job of the
468,750-particle twin in the full-size parity tests."""
import time

import numpy as np
import pytest
import torch

import oracle
from paper_1206_0115_amd import fmm, inputs

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# The FMM's own error against exact sums at the 30M workload's density and
# order (the order-10 interpolation, with the SVD truncation at the
# workload's tolerance), measured on its 469k-particle twin; the mixed mode
# adds at most the 5e-7 the twin's gate tests allow.
TWIN_FP64_VS_EXACT = 8e-6


def test_twin_fmm_error_against_exact_sums():
    kind, n, h, l, seed = inputs.CONFIGS["cube469k_h7_p10"]
    print("469k order-10 twin against exact sums", flush=True)
    pos, q = inputs.make(kind, n, seed)
    idx = np.sort(np.random.default_rng(11).choice(n, 256, replace=False))
    pd, fd = oracle.direct_sampled(pos, q, idx)
    plan = fmm.Plan(torch.from_numpy(pos).cuda(), h, l, "fp64",
                    m2l_tolerance=inputs.SVD_TOL["cube469k_h7_p10"])
    errs = {}
    for mode in ("fp64", "fp64_svd", "mixed_svd"):
        plan.set_precision(mode)
        phi, f = plan.evaluate(torch.from_numpy(q).cuda())
        torch.cuda.synchronize()
        phi, f = phi.cpu().numpy()[idx], f.cpu().numpy()[idx]
        errs[mode] = max(rel(phi, pd), rel(f, fd))
        print(f"  {mode}: phi {rel(phi, pd):.3e} F {rel(f, fd):.3e}", flush=True)
    assert errs["fp64"] <= TWIN_FP64_VS_EXACT
    assert errs["fp64_svd"] <= TWIN_FP64_VS_EXACT
    assert errs["mixed_svd"] <= TWIN_FP64_VS_EXACT + 5e-7


def test_cube30m_order10_mixed_compressed():
    kind, n, h, l, seed = inputs.CONFIGS["cube30m_h9_p10"]
    print("30M order-10 cube, mixed_svd", flush=True)
    pos, q = inputs.make(kind, n, seed)
    pos_d, q_d = torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda()
    t0 = time.perf_counter()
    plan = fmm.Plan(pos_d, h, l, "mixed_svd", m2l_tolerance=inputs.SVD_TOL["cube30m_h9_p10"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    inf = plan.info()
    print(f"  plan {t1 - t0:.1f} s, {inf.device_bytes / 1e9:.1f} GB, leaves {inf.n_leaf}, "
          f"far pairs {inf.far_pairs}", flush=True)
    assert inf.n_leaf > 13_000_000 and inf.far_pairs > 2_000_000_000
    assert inf.device_bytes < 260e9
    phi, f = plan.evaluate(q_d)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    phi, f = phi.cpu().numpy(), f.cpu().numpy()
    print(f"  evaluate {t2 - t1:.1f} s", flush=True)
    plan.release()
    del pos_d, q_d
    idx = np.sort(np.random.default_rng(11).choice(n, 256, replace=False))
    pd, fd = oracle.direct_sampled(pos, q, idx)
    e = max(rel(phi[idx], pd), rel(f[idx], fd))
    print(f"  rel L2 vs exact direct sum at 256 targets {e:.3e}", flush=True)
    assert np.isfinite(phi).all() and np.isfinite(f).all()
    assert e <= TWIN_FP64_VS_EXACT + 5e-7
