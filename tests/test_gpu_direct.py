"""Exact sums at sampled targets on the GPU (fmm_direct_sampled, Eq. 1-2)
against the oracle's direct summation: FP64, so within rounding (1e-13
relative L2); bit-identical from call to call; zero-distance pairs skipped;
an out-of-range target index gives NaN for that target only."""
import numpy as np
import pytest
import torch

import oracle
from paper_1206_0115_amd import fmm, inputs

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("kind,n,nt,kernel", [
    ("cube", 50_000, 300, "inv_r"),       # several chunks, ragged target tile
    ("sphere", 70_001, 65, "inv_r2"),
    ("cube", 1, 1, "inv_r"),              # a lone particle: nothing to sum
    ("cube", 777, 777, "inv_r"),          # every particle a target
])
def test_direct_sampled_matches_oracle(kind, n, nt, kernel):
    print(f"direct {kind} n={n} nt={nt} {kernel}", flush=True)
    pos, q = inputs.make(kind, n, 61)
    idx = np.sort(np.random.default_rng(3).choice(n, nt, replace=False)).astype(np.int64)
    phi, f = fmm.direct_sampled(dev(pos), dev(q), dev(idx), kernel=kernel)
    torch.cuda.synchronize()
    p_o, f_o = oracle.direct_sampled(pos, q, idx, kernel=1 if kernel == "inv_r" else 2)
    phi, f = phi.cpu().numpy(), f.cpu().numpy()
    if n == 1:
        assert phi[0] == 0.0 and not f.any()
        return
    assert rel(phi, p_o) <= 1e-13 and rel(f, f_o) <= 1e-13
    phi2, f2 = fmm.direct_sampled(dev(pos), dev(q), dev(idx), kernel=kernel)
    assert np.array_equal(phi2.cpu().numpy(), phi) and np.array_equal(f2.cpu().numpy(), f)


def test_direct_sampled_coincident_and_bad_targets():
    pos = np.full((40, 3), 0.5)
    pos[20:] = 0.25
    q = np.linspace(-1.0, 1.0, 40)
    idx = np.array([0, 39, 40, -1], dtype=np.int64)
    phi, f = fmm.direct_sampled(dev(pos), dev(q), dev(idx))
    phi, f = phi.cpu().numpy(), f.cpu().numpy()
    p_o, f_o = oracle.direct_sampled(pos, q, idx[:2])
    np.testing.assert_allclose(phi[:2], p_o, rtol=1e-14)
    np.testing.assert_allclose(f[:2], f_o, rtol=1e-14)
    assert np.isnan(phi[2:]).all() and np.isnan(f[2:]).all()
