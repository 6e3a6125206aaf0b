"""Pins of the oracle's operators and whole FMM.

Operators: conservation of charge and dipole, exact translation identities
(M2M after P2M of the children equals P2M of the parent; L2P after L2L equals
L2P of the parent), the M2L matrix against 1/r between node positions built
here from cell centres, its symmetry and homogeneity, and the far-field chain
P2M -> M2L -> L2P against the exact interaction of two separated clusters.

Whole FMM: one level is bit-exact with the direct sum; two levels have no far
field and agree to rounding; the error against the direct sum falls strictly
with the order.
"""
import itertools

import numpy as np
import pytest

from paper_1206_0115_amd import inputs


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def points_in_box(rng, n, c, a):
    return c + a * rng.uniform(-1, 1, (n, 3))


@pytest.mark.parametrize("l", [1, 2, 4, 7])
def test_p2m_conserves_charge_and_dipole(orc, l):
    rng = np.random.default_rng(l)
    c, a = np.array([0.3, -0.2, 0.9]), 0.125
    x = points_in_box(rng, 40, c, a)
    q = rng.uniform(-1, 1, 40)
    W = orc.p2m(l, x, q, c, a).reshape(l, l, l)
    assert W.sum() == pytest.approx(q.sum(), abs=1e-13)
    if l >= 2:
        xi = orc.cheb_nodes(l)
        u = (x - c) / a
        for d in range(3):
            shape = [1, 1, 1]
            shape[d] = l
            assert (W * xi.reshape(shape)).sum() == pytest.approx((q * u[:, d]).sum(), abs=1e-13)


@pytest.mark.parametrize("l", [2, 3, 5, 7])
def test_m2m_of_children_equals_parent_p2m(orc, l):
    rng = np.random.default_rng(10 + l)
    cp, ap = np.array([0.5, 0.5, 0.5]), 0.5
    x = points_in_box(rng, 200, cp, ap)
    q = rng.uniform(-1, 1, 200)
    Wp_direct = orc.p2m(l, x, q, cp, ap)
    Wp = np.zeros(l ** 3)
    ac = ap / 2
    for o in range(8):
        sig = np.array([1 if (o >> d) & 1 else -1 for d in range(3)])
        cc = cp + sig * ac
        inside = np.all(np.sign(x - cp) == sig, axis=1)
        Wc = orc.p2m(l, x[inside], q[inside], cc, ac)
        Wp = orc.m2m(l, o, Wc, Wp)
    assert np.max(np.abs(Wp - Wp_direct)) <= 1e-13 * max(1.0, np.abs(Wp_direct).max())


@pytest.mark.parametrize("l", [2, 4, 6])
def test_l2p_of_l2l_equals_parent_l2p(orc, l):
    rng = np.random.default_rng(20 + l)
    Lp = rng.standard_normal(l ** 3)
    cp, ap = np.array([-1.0, 2.0, 0.25]), 0.5
    ac = ap / 2
    for o in (0, 3, 5, 6):
        sig = np.array([1 if (o >> d) & 1 else -1 for d in range(3)])
        cc = cp + sig * ac
        x = points_in_box(rng, 25, cc, ac)
        q = rng.uniform(-1, 1, 25)
        Lc = orc.l2l(l, o, Lp)
        phi_c, f_c = orc.l2p(l, x, q, cc, ac, Lc)
        phi_p, f_p = orc.l2p(l, x, q, cp, ap, Lp)
        np.testing.assert_allclose(phi_c, phi_p, atol=1e-12 * np.abs(phi_p).max())
        np.testing.assert_allclose(f_c, f_p, atol=1e-11 * np.abs(f_p).max())


def test_l2p_gradient_matches_finite_difference(orc):
    # F = -q grad(phi): compare with a central difference of the L2P potential
    l, c, a = 5, np.array([0.0, 0.0, 0.0]), 0.25
    rng = np.random.default_rng(3)
    Loc = rng.standard_normal(l ** 3)
    x = points_in_box(rng, 6, c, 0.8 * a)
    q = rng.uniform(0.5, 1.5, 6)
    phi, f = orc.l2p(l, x, q, c, a, Loc)
    e = 1e-6
    for d in range(3):
        dx = np.zeros(3)
        dx[d] = e
        pp, _ = orc.l2p(l, x + dx, q, c, a, Loc)
        pm, _ = orc.l2p(l, x - dx, q, c, a, Loc)
        np.testing.assert_allclose(f[:, d], -q * (pp - pm) / (2 * e), rtol=1e-6, atol=1e-6)


def node_positions(orc, l, c, a):
    xi = orc.cheb_nodes(l)
    g = np.stack(np.meshgrid(xi, xi, xi, indexing="ij"), -1).reshape(-1, 3)
    return c + a * g


@pytest.mark.parametrize("t", [(2, 0, 0), (-3, 1, 2), (0, -2, 3), (3, 3, -3)])
def test_m2l_matrix_is_kernel_between_nodes(orc, t):
    l, w = 4, 0.125
    a = w / 2
    ct = np.array([0.1, 0.2, 0.3])
    cs = ct + w * np.array(t)
    K = orc.m2l_matrix(l, a, w, t)
    xm = node_positions(orc, l, ct, a)
    yn = node_positions(orc, l, cs, a)
    ref = 1.0 / np.linalg.norm(xm[:, None, :] - yn[None, :, :], axis=2)
    np.testing.assert_allclose(K, ref, rtol=1e-13)


def test_m2l_symmetry_and_homogeneity(orc):
    l = 3
    xi = orc.cheb_nodes(l)
    t = np.array([3, -2, 1])
    K = orc.m2l_matrix(l, 0.5, 1.0, t)
    idx = np.array(list(itertools.product(range(l), repeat=3)))
    for p in itertools.permutations(range(3)):
        for s in itertools.product((1, -1), repeat=3):
            gt = np.array([s[d] * t[p[d]] for d in range(3)])
            Kg = orc.m2l_matrix(l, 0.5, 1.0, gt)
            # node m maps to g(m): axis d takes m_{p(d)}, mirrored if s_d < 0
            gm = np.array([[m[p[d]] if s[d] > 0 else l - 1 - m[p[d]] for d in range(3)]
                           for m in idx])
            flat = (gm[:, 0] * l + gm[:, 1]) * l + gm[:, 2]
            np.testing.assert_allclose(Kg[np.ix_(flat, flat)], K, rtol=1e-15)
    # 1/r is homogeneous of degree -1
    K2 = orc.m2l_matrix(l, 0.125, 0.25, t)
    np.testing.assert_allclose(K2, 4.0 * K, rtol=1e-15)
    assert np.all(np.abs(xi) < 1)


@pytest.mark.parametrize("t", [(2, 0, 0), (3, -2, 1)])
def test_far_chain_approximates_exact_interaction(orc, t):
    # P2M in the source cell, M2L, L2P in the target cell against the exact
    # sum between the two clusters: the error falls with the order
    rng = np.random.default_rng(5)
    w = 0.25
    a = w / 2
    ct = np.array([0.0, 0.0, 0.0])
    cs = ct + w * np.array(t)
    xs, xt = points_in_box(rng, 60, cs, a), points_in_box(rng, 50, ct, a)
    qs, qt = rng.uniform(-1, 1, 60), rng.uniform(-1, 1, 50)
    pos = np.vstack([xt, xs])
    q = np.concatenate([qt, np.zeros(60)])
    q2 = np.concatenate([qt, qs])
    # exact potential at targets from sources only: direct over all minus
    # direct with the sources' charges zeroed
    pd_all, fd_all = orc.direct(pos, q2)
    pd_t, fd_t = orc.direct(pos, q)
    pe, fe = (pd_all - pd_t)[:50], (fd_all - fd_t)[:50]
    errs = []
    for l in (2, 3, 4, 5, 6, 7, 8):
        W = orc.p2m(l, xs, qs, cs, a)
        Loc = orc.m2l_matrix(l, a, w, t) @ W
        p, f = orc.l2p(l, xt, qt, ct, a, Loc)
        errs.append(max(rel(p, pe), rel(f, fe)))
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-3 * errs[0], errs


def test_one_level_is_bit_exact_with_direct(orc):
    pos, q = inputs.uniform_cube(700, 31)
    pd, fd = orc.direct(pos, q)
    p, f, pn, fn, pf, ff = orc.Tree(pos, 1).fmm(5, q, parts=True)
    assert np.array_equal(p, pd) and np.array_equal(f, fd)
    assert not pf.any() and not ff.any()


@pytest.mark.parametrize("kind", ["cube", "sphere"])
def test_two_levels_equal_direct(orc, kind):
    pos, q = inputs.make(kind, 900, 32)
    pd, fd = orc.direct(pos, q)
    p, f, pn, fn, pf, ff = orc.Tree(pos, 2).fmm(4, q, parts=True)
    assert not pf.any() and not ff.any()
    assert rel(p, pd) < 1e-14 and rel(f, fd) < 1e-14


@pytest.mark.parametrize("kind,n,h,orders", [
    ("cube", 3000, 3, range(2, 10)),
    ("cube", 3000, 4, range(2, 9)),
    ("sphere", 4000, 5, range(2, 8)),
])
def test_error_falls_strictly_with_order(orc, kind, n, h, orders):
    pos, q = inputs.make(kind, n, 33)
    pd, fd = orc.direct(pos, q)
    t = orc.Tree(pos, h)
    errs = []
    for l in orders:
        p, f = t.fmm(l, q)
        errs.append(max(rel(p, pd), rel(f, fd)))
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:])), errs
    assert errs[-1] < 2e-6, errs


def test_sampled_fmm_equals_full_bitwise(orc):
    pos, q = inputs.uniform_cube(5000, 34)
    t = orc.Tree(pos, 4)
    p, f = t.fmm(4, q)
    idx = np.array([17, 4999, 0, 2500, 17])
    ps, fs = t.fmm(4, q, targets=idx)
    assert np.array_equal(ps, p[idx]) and np.array_equal(fs, f[idx])


def test_near_plus_far_is_the_output(orc):
    pos, q = inputs.sphere_surface(3000, 35)
    p, f, pn, fn, pf, ff = orc.Tree(pos, 5).fmm(3, q, parts=True)
    assert np.array_equal(p, pn + pf) and np.array_equal(f, fn + ff)
