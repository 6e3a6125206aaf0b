"""The mutual near field (the reduction form of P2P, Sec. 5): each pair of
distinct neighbour leaves is computed once and its terms go to both leaves.

The pair lists are checked against the oracle's tree: every unordered pair of
distinct neighbour leaves appears exactly once, in the list of its forward
near slot and of the colour of its first leaf, and no two pairs of one list
share a leaf (what lets one launch update both leaves without atomics).  The
near part matches the oracle's (FP64 within 1e-12; the mixed modes within the
1e-6 gate of their FP64 runs), so does the total, and results are
deterministic and equal across schedules and graph replay."""
import numpy as np
import pytest
import torch

import oracle
from paper_1206_0115_amd import fmm, inputs

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
MIXED_GATE = 1e-6


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def say(msg):
    print(msg, flush=True)


def leaf_coords(keys, bits):
    """Grid coordinates of Morton keys (x in bit 3b, y in 3b+1, z in 3b+2)."""
    keys = keys.astype(np.uint64)
    c = np.zeros((len(keys), 3), dtype=np.int64)
    for b in range(bits):
        for d in range(3):
            c[:, d] |= ((keys >> np.uint64(3 * b + d)) & np.uint64(1)).astype(np.int64) << b
    return c


def expected_lists(tree, h):
    """The 26 lists by their definition: list 2k + c holds the leaves a whose
    neighbour at slot s = 14 + k (offset (s//9 - 1, s//3 % 3 - 1, s % 3 - 1))
    exists and whose coordinate along the offset's first non-zero axis has
    parity c."""
    c = leaf_coords(tree.cell_keys(h - 1), h - 1)
    where = {tuple(x): i for i, x in enumerate(c.tolist())}
    lists = [[] for _ in range(26)]
    pairs = [[] for _ in range(26)]
    for k in range(13):
        s = 14 + k
        o = np.array([s // 9 - 1, s // 3 % 3 - 1, s % 3 - 1])
        axis = int(np.flatnonzero(o)[0])
        for a, x in enumerate(c.tolist()):
            b = where.get(tuple(np.array(x) + o))
            if b is not None:
                lists[2 * k + (x[axis] & 1)].append(a)
                pairs[2 * k + (x[axis] & 1)].append((a, b))
    return lists, pairs


LIST_CASES = [("cube", 20000, 4, 31), ("sphere", 30000, 5, 32), ("cube", 700, 6, 33),
              ("cube", 3000, 2, 34), ("cube", 3000, 1, 35)]


@pytest.mark.parametrize("kind,n,h,seed", LIST_CASES)
def test_pair_lists_partition_the_neighbour_pairs(kind, n, h, seed):
    say(f"mutual lists {kind} n={n} h={h}")
    pos, _ = inputs.make(kind, n, seed)
    plan = fmm.Plan(dev(pos), h, 3)
    with pytest.raises(fmm.FMMError):
        plan.export(fmm.EXPORT_MUTUAL_OFF)  # not built before the first switch
    plan.set_near("mutual")
    off = plan.export(fmm.EXPORT_MUTUAL_OFF)
    idx = plan.export(fmm.EXPORT_MUTUAL_IDX)
    tree = oracle.Tree(pos, h)
    lists, pairs = expected_lists(tree, h)
    assert off[0] == 0 and np.all(np.diff(off) >= 0)
    for k in range(26):
        assert idx[off[k]:off[k + 1]].tolist() == lists[k], k
        touched = [x for pr in pairs[k] for x in pr]
        assert len(set(touched)) == len(touched), k  # the list's pairs share no leaf
    # every unordered pair of distinct neighbour leaves exactly once
    noff, nidx = tree.near()
    want = {(min(a, int(b)), max(a, int(b))) for a in range(tree.n_leaf)
            for b in nidx[noff[a]:noff[a + 1]] if int(b) != a}
    got = [(min(a, b), max(a, b)) for pr in pairs for a, b in pr]
    assert len(got) == len(set(got)) and set(got) == want


PARITY = [
    ("cube", 20000, 4, 4, 1001),
    ("sphere", 30000, 5, 5, 14),
    ("sphere", 60000, 4, 3, 17),   # about 250 particles per leaf: several chunks per side
    ("cube", 5000, 2, 4, 16),      # 625 per leaf
    ("cube", 700, 6, 3, 15),       # mostly one particle per leaf
    ("cube", 3000, 1, 4, 11),      # one leaf: no pairs of distinct leaves
]


@pytest.mark.parametrize("kernel", ["inv_r", "inv_r2"])
@pytest.mark.parametrize("kind,n,h,l,seed", PARITY)
def test_mutual_near_field_matches_oracle(kind, n, h, l, seed, kernel):
    say(f"mutual parity {kind} n={n} h={h} l={l} {kernel}")
    pos, q = inputs.make(kind, n, seed)
    kp = fmm.KERNELS[kernel]
    tree = oracle.Tree(pos, h)
    p_o, f_o, pn_o, fn_o, _, _ = tree.fmm(l, q, parts=True, kernel=kp)
    plan = fmm.Plan(dev(pos), h, l, "fp64")
    plan.set_kernel(kernel)
    qd = dev(q)
    res = {}
    for mode in ("fp64", "mixed"):
        plan.set_precision(mode)
        for near in ("one_sided", "mutual"):
            plan.set_near(near)
            pn, fn, _, _ = plan.evaluate_parts(qd)
            phi, f = plan.evaluate(qd)
            torch.cuda.synchronize()
            res[mode, near] = [host(t) for t in (pn, fn, phi, f)]
    pn, fn, phi, f = res["fp64", "mutual"]
    if h >= 2 and n >= 5000:  # many pairs of distinct leaves: the mutual form ran (another summation order)
        assert not np.array_equal(fn, res["fp64", "one_sided"][1])
    assert rel(pn, pn_o) <= FP64_TOL, rel(pn, pn_o)
    assert rel(fn, fn_o) <= FP64_TOL, rel(fn, fn_o)
    assert rel(phi, p_o) <= FP64_TOL and rel(f, f_o) <= FP64_TOL
    ref = res["fp64", "one_sided"]
    for a, b in zip(res["mixed", "mutual"], ref):
        assert rel(a, b) <= MIXED_GATE, rel(a, b)
    # the near part of the mixed mutual form errs no more than the one-sided
    # one (both round the pair differences once and fold per chunk or leaf)
    e_mut = rel(res["mixed", "mutual"][1], ref[1])
    e_one = rel(res["mixed", "one_sided"][1], ref[1])
    say(f"  mixed near-force error: mutual {e_mut:.2e}, one-sided {e_one:.2e}")
    assert e_mut <= 2 * e_one + 1e-9


@pytest.mark.parametrize("n", [1, 2, 3, 40])
def test_tiny_inputs_and_coincident_particles(n):
    say(f"mutual tiny n={n}")
    pos, q = inputs.uniform_cube(n, 36)
    if n == 40:
        pos[20:] = pos[0]  # half the particles at one point (one leaf)
    for h in (1, 3, 5):
        plan = fmm.Plan(dev(pos), h, 3, "fp64")
        plan.set_near("mutual")
        phi, f = plan.evaluate(dev(q))
        torch.cuda.synchronize()
        p_o, f_o = oracle.Tree(pos, h).fmm(3, q)
        assert np.allclose(host(phi), p_o, rtol=1e-12, atol=1e-12 * np.abs(p_o).max())
        assert np.allclose(host(f), f_o, rtol=1e-12, atol=1e-12 * np.abs(f_o).max())


@pytest.mark.parametrize("mode", ["fp64", "mixed_svd"])
def test_mutual_deterministic_across_schedules_and_graph(mode):
    say(f"mutual schedules and graph {mode}")
    pos, q = inputs.sphere_surface(50000, 37)
    q2 = np.random.default_rng(38).uniform(-1.0, 1.0, len(q))
    plan = fmm.Plan(dev(pos), 5, 5, mode)
    plan.set_near("mutual")
    qs = [dev(q), dev(q2)]
    plan.set_schedule("serial")
    ref = [[host(t) for t in plan.evaluate(qq)] for qq in qs]
    for sched in ("forked", "pipelined"):
        plan.set_schedule(sched)
        outs = [plan.evaluate(qs[k % 2]) for k in range(3)]  # queued back to back
        torch.cuda.synchronize()
        for k, (phi, f) in enumerate(outs):
            assert np.array_equal(host(phi), ref[k % 2][0]), (sched, k)
            assert np.array_equal(host(f), ref[k % 2][1]), (sched, k)
        plan.set_graph(True)
        for k in range(4):
            phi, f = plan.evaluate(qs[k % 2])
            torch.cuda.synchronize()
            assert np.array_equal(host(phi), ref[k % 2][0]), (sched, "graph", k)
            assert np.array_equal(host(f), ref[k % 2][1]), (sched, "graph", k)
            x = torch.randn(256, 256, device="cuda")  # eager work between replays
            (x @ x).sum().item()
        plan.set_graph(False)
    # back to one-sided: the graph of the mutual form is not replayed for it
    plan.set_schedule("serial")
    plan.set_graph(True)
    plan.set_near("one_sided")
    phi, f = plan.evaluate(qs[0])
    plan.set_graph(False)
    phi1, f1 = plan.evaluate(qs[0])
    torch.cuda.synchronize()
    assert np.array_equal(host(phi), host(phi1)) and np.array_equal(host(f), host(f1))
    assert rel(host(phi1), ref[0][0]) <= (1e-13 if mode == "fp64" else MIXED_GATE)
