"""GPU parity against the oracle, through the C-ABI.

Plan data (Morton keys, permutation, leaf offsets, cell keys, near and far
lists) must be bit-exact; FP64 potentials and forces within 1e-12 relative L2
(the bound the FMM's FP64 path is held to), separately for the near field, the
far field and their sum.  Full-size configurations are checked on a seeded
sample of targets that the oracle evaluates one by one.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1206_0115_amd import fmm, inputs

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a - b)


def say(msg):
    print(msg, flush=True)


def check_plan(plan, tree):
    h = tree.h
    assert np.array_equal(plan.export(fmm.EXPORT_KEYS), tree.keys())
    assert np.array_equal(plan.export(fmm.EXPORT_PERM), tree.perm())
    assert np.array_equal(plan.export(fmm.EXPORT_LEAF_START), tree.leaf_start())
    inf = plan.info()
    assert inf.n_leaf == tree.n_leaf
    assert list(inf.ncell)[:h] == tree.ncell
    for lv in range(h):
        assert np.array_equal(plan.export(fmm.EXPORT_CELL_KEYS, lv), tree.cell_keys(lv))
    off, idx = tree.near()
    assert np.array_equal(plan.export(fmm.EXPORT_NEAR_OFF), off)
    assert np.array_equal(plan.export(fmm.EXPORT_NEAR_IDX), idx)
    tot = 0
    for lv in range(2, h):
        off, idx = tree.far(lv)
        assert np.array_equal(plan.export(fmm.EXPORT_FAR_OFF, lv), off), lv
        assert np.array_equal(plan.export(fmm.EXPORT_FAR_IDX, lv), idx), lv
        assert inf.far_pairs_level[lv] == len(idx)
        tot += len(idx)
    assert inf.far_pairs == tot
    assert np.array_equal(np.array(tree.lo), np.array(inf.lo)) and inf.L == tree.L


SMALL = [
    ("cube", 20000, 4, 5, 1001),   # the 20k-particle configuration
    ("cube", 3000, 1, 4, 11),
    ("cube", 3000, 2, 4, 12),
    ("cube", 3000, 3, 6, 13),
    ("sphere", 6000, 5, 4, 14),
    ("cube", 700, 6, 3, 15),       # ragged: mostly 1-particle leaves
    ("cube", 5000, 2, 2, 16),      # >64 particles per leaf: several target passes
    ("sphere", 4000, 4, 8, 17),
    ("cube", 2500, 4, 1, 18),
    ("cube", 1500, 3, 12, 19),     # largest supported order
]


@pytest.mark.parametrize("kind,n,h,l,seed", SMALL)
def test_plan_bit_exact(kind, n, h, l, seed):
    say(f"plan parity {kind} n={n} h={h} l={l}")
    pos, _ = inputs.make(kind, n, seed)
    plan = fmm.Plan(dev(pos), h, l)
    check_plan(plan, oracle.Tree(pos, h))


@pytest.mark.parametrize("kind,n,h,l,seed", SMALL)
def test_fp64_parity(kind, n, h, l, seed):
    say(f"fp64 parity {kind} n={n} h={h} l={l}")
    pos, q = inputs.make(kind, n, seed)
    plan = fmm.Plan(dev(pos), h, l)
    tree = oracle.Tree(pos, h)
    p_o, f_o, pn_o, fn_o, pf_o, ff_o = tree.fmm(l, q, parts=True)
    phi, f = plan.evaluate(dev(q))
    torch.cuda.synchronize()
    assert rel(host(phi), p_o) <= FP64_TOL, rel(host(phi), p_o)
    assert rel(host(f), f_o) <= FP64_TOL, rel(host(f), f_o)
    pn, fn, pf, ff = plan.evaluate_parts(dev(q))
    torch.cuda.synchronize()
    assert rel(host(pn), pn_o) <= FP64_TOL
    assert rel(host(fn), fn_o) <= FP64_TOL
    if h >= 3:
        assert rel(host(pf), pf_o) <= FP64_TOL, rel(host(pf), pf_o)
        assert rel(host(ff), ff_o) <= FP64_TOL, rel(host(ff), ff_o)
    else:
        assert not host(pf).any() and not host(ff).any()


# Orders whose l^2 lines take two or three rounds of a wavefront in the
# transfer passes (l >= 9), over two and three levels of M2M and L2L, with
# dense leaves (lanes over particles in L2P) and sparse ones (lanes over the
# l^3 terms), against the oracle at sampled targets.
HIGH = [(h, l, n) for l in (9, 10, 11, 12) for h, n in ((4, 30000), (5, 60000))] + [
    (5, 9, 5000), (4, 11, 2000)]


@pytest.mark.parametrize("h,l,n", HIGH)
def test_high_order_transfer_levels(h, l, n):
    say(f"high-order transfer levels h={h} l={l} n={n}")
    pos, q = inputs.make("cube", n, 91)
    tree = oracle.Tree(pos, h)
    idx = np.sort(np.random.default_rng(3).choice(n, 32, replace=False))
    p_o, f_o = tree.fmm(l, q, targets=idx)
    plan = fmm.Plan(dev(pos), h, l, "fp64")
    phi, f = plan.evaluate(dev(q))
    torch.cuda.synchronize()
    assert rel(host(phi)[idx], p_o) <= FP64_TOL
    assert rel(host(f)[idx], f_o) <= FP64_TOL


def test_one_level_matches_direct():
    pos, q = inputs.uniform_cube(2000, 21)
    plan = fmm.Plan(dev(pos), 1, 5)
    phi, f = plan.evaluate(dev(q))
    pd, fd = oracle.direct(pos, q)
    assert rel(host(phi), pd) <= 1e-14 and rel(host(f), fd) <= 1e-14


@pytest.mark.parametrize("n", [1, 2, 3])
def test_tiny_inputs(n):
    say(f"tiny n={n}")
    pos, q = inputs.uniform_cube(n, 22)
    for h in (1, 3, 5):
        plan = fmm.Plan(dev(pos), h, 4)
        phi, f = plan.evaluate(dev(q))
        pd, fd = oracle.Tree(pos, h).fmm(4, q)
        np.testing.assert_allclose(host(phi), pd, rtol=1e-13, atol=0)
        np.testing.assert_allclose(host(f), fd, rtol=1e-12, atol=1e-300)


def test_coincident_particles():
    pos = np.full((50, 3), 0.25)
    q = np.linspace(-1, 1, 50)
    plan = fmm.Plan(dev(pos), 4, 3)
    phi, f = plan.evaluate(dev(q))
    assert not host(phi).any() and not host(f).any()
    assert plan.info().L == 1.0 and plan.info().n_leaf == 1


def test_non_finite_positions_rejected():
    pos, _ = inputs.uniform_cube(100, 23)
    pos[17, 1] = np.nan
    with pytest.raises(fmm.FMMError) as e:
        fmm.Plan(dev(pos), 3, 4)
    assert e.value.code == fmm.FMM_ERR_ARG
    pos[17, 1] = np.inf
    with pytest.raises(fmm.FMMError):
        fmm.Plan(dev(pos), 3, 4)


def test_deterministic_and_reusable():
    pos, q = inputs.sphere_surface(8000, 24)
    plan = fmm.Plan(dev(pos), 5, 5)
    a = [host(t) for t in plan.evaluate(dev(q))]
    q2 = np.random.default_rng(0).uniform(-1, 1, len(q))
    plan.evaluate(dev(q2))
    b = [host(t) for t in plan.evaluate(dev(q))]
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


# (name, sampled targets, bound on the dense mixed mode against FP64): the
# 1e-6 gate everywhere.  The FP32 M2L accumulates Chebyshev coefficients,
# so its rounding no longer reaches the forces through the gradient of the
# order-10 interpolant (4.0e-6 when it accumulated node values; 3.4e-7 now
# on the order-10 twin).
FULL = [
    ("cube1m_h6_p7", 96, 1e-6),
    ("sphere10m_h8_p7", 96, 1e-6),
    ("cube469k_h7_p10", 48, 1e-6),  # density twin of the 30M, order-10 cube
]


@pytest.mark.parametrize("name,samples,mixed_bound", FULL)
def test_full_size_sampled_parity(name, samples, mixed_bound):
    kind, n, h, l, seed = inputs.CONFIGS[name]
    say(f"full-size sampled parity {name}")
    pos, q = inputs.make(kind, n, seed)
    plan = fmm.Plan(dev(pos), h, l)
    tree = oracle.Tree(pos, h)
    check_plan(plan, tree)
    phi, f = plan.evaluate(dev(q))
    torch.cuda.synchronize()
    idx = np.sort(np.random.default_rng(7).choice(n, samples, replace=False))
    p_o, f_o = tree.fmm(l, q, targets=idx)
    assert rel(host(phi)[idx], p_o) <= FP64_TOL
    assert rel(host(f)[idx], f_o) <= FP64_TOL
    # the same launch in the mixed mode, against the FP64 path: the gate
    plan.set_precision("mixed")
    phm, fm = plan.evaluate(dev(q))
    torch.cuda.synchronize()
    e = max(rel(host(phm), host(phi)), rel(host(fm), host(f)))
    say(f"  mixed vs fp64 rel L2 {e:.3e}")
    assert e <= mixed_bound


def test_second_stream_while_in_flight_is_refused():
    """A plan evaluated on one stream refuses an evaluation on another stream
    (FMM_ERR_STATE) until the first has finished; then it is accepted."""
    pos, q = inputs.uniform_cube(200_000, 31)
    plan = fmm.Plan(dev(pos), 5, 7)
    qd = dev(q)
    a, b = torch.cuda.Stream(), torch.cuda.Stream()
    out = plan.evaluate(qd, stream=a)
    a.synchronize()
    ref = [host(t) for t in out]
    x = torch.rand(4096, 4096, dtype=torch.float64, device="cuda")
    with torch.cuda.stream(a):
        for _ in range(4):  # keep stream a busy (about 10 ms) ahead of the evaluation
            x = torch.matmul(x, x) * 1e-3
    plan.evaluate(qd, stream=a)
    with pytest.raises(fmm.FMMError) as e:
        plan.evaluate(qd, stream=b)
    assert e.value.code == fmm.FMM_ERR_STATE
    a.synchronize()
    phi, f = plan.evaluate(qd, stream=b)
    b.synchronize()
    assert np.array_equal(host(phi), ref[0]) and np.array_equal(host(f), ref[1])


def test_bf16_mode_is_refused():
    pos, _ = inputs.uniform_cube(1000, 32)
    plan = fmm.Plan(dev(pos), 3, 4, "mixed")
    with pytest.raises(fmm.FMMError) as e:
        plan.set_precision("mixed_bf16")
    assert e.value.code == fmm.FMM_ERR_ARG and "BF16" in str(e.value)
    assert plan.info().precision == fmm.FMM_MIXED_FP32
