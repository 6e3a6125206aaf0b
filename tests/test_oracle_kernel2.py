"""Pins of the oracle for the second kernel P(x, y) = 1/|x - y|^2.

The black-box scheme (Sec. 2.1) needs only point evaluations of the kernel;
1/r^2 is homogeneous of degree -2, so its unit M2L operators scale by a^-2
per level.  Force convention as for 1/r: F_i = -q_i grad phi(x_i) =
q_i sum_j q_j 2 (x_i - x_j) / r^4.  Each check below is fixed by the
mathematics, not by the oracle's code.
"""
import numpy as np
import pytest

from paper_1206_0115_amd import inputs

K2 = 2


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_two_particle_closed_form(orc):
    pos = np.array([[0.0, 0.0, 0.0], [3.0, 4.0, 0.0]])
    q = np.array([2.0, -0.5])
    phi, f = orc.direct(pos, q, kernel=K2)
    # r^2 = 25: phi_0 = q_1/25, phi_1 = q_0/25; F_0 = 2 q_0 q_1 (x_0-x_1)/625
    assert phi[0] == pytest.approx(-0.02, rel=1e-15)
    assert phi[1] == pytest.approx(0.08, rel=1e-15)
    np.testing.assert_allclose(f[0], [6 / 625, 8 / 625, 0.0], rtol=1e-15, atol=0)
    np.testing.assert_allclose(f[1], [-6 / 625, -8 / 625, 0.0], rtol=1e-15, atol=0)


def test_cube_vertices_closed_form(orc):
    # unit charges on the unit cube's vertices: 3 neighbours at r^2 = 1, 3 at
    # 2, 1 at 3; the force is along the outward diagonal with components
    # 2 (1 + 2 * 1/4 + 1/9)
    v = np.array([[i, j, k] for i in (0, 1) for j in (0, 1) for k in (0, 1)], float)
    phi, f = orc.direct(v, np.ones(8), kernel=K2)
    np.testing.assert_allclose(phi, 3 + 3 / 2 + 1 / 3, rtol=1e-15)
    np.testing.assert_allclose(f, (2 * v - 1) * 2 * (1 + 0.5 + 1 / 9), rtol=1e-14,
                               atol=1e-15)


def test_forces_sum_to_zero_and_dilation(orc):
    pos, q = inputs.uniform_cube(2000, 81)
    phi, f = orc.direct(pos, q, kernel=K2)
    assert np.abs(f.sum(axis=0)).max() < 1e-11 * np.abs(f).sum()
    s = 0.25  # a power of two: the scaled positions are exact
    phi_s, f_s = orc.direct(pos * s, q, kernel=K2)
    np.testing.assert_allclose(phi_s, phi / s ** 2, rtol=1e-13)
    np.testing.assert_allclose(f_s, f / s ** 3, rtol=1e-13, atol=1e-9)


def test_force_is_minus_q_grad_phi(orc):
    pos, q = inputs.uniform_cube(200, 82)
    _, f = orc.direct(pos, q, kernel=K2)
    i, h = 17, 1e-6
    g = np.empty(3)
    for d in range(3):
        pp, pm = pos.copy(), pos.copy()
        pp[i, d] += h
        pm[i, d] -= h
        # potential at particle i from all others, i moved
        g[d] = (orc.direct(pp, q, kernel=K2)[0][i] - orc.direct(pm, q, kernel=K2)[0][i]) / (2 * h)
    np.testing.assert_allclose(f[i], -q[i] * g, rtol=1e-6)


def test_sampled_direct_matches_full(orc):
    pos, q = inputs.sphere_surface(1500, 83)
    phi, f = orc.direct(pos, q, kernel=K2)
    idx = np.array([0, 7, 1499, 7])
    ps, fs = orc.direct_sampled(pos, q, idx, kernel=K2)
    assert np.array_equal(ps, phi[idx]) and np.array_equal(fs, f[idx])


@pytest.mark.parametrize("t", [(2, 0, 0), (3, -2, 1), (-3, -3, -3)])
def test_m2l_matrix_is_kernel_between_nodes(orc, t):
    l, a, w = 3, 0.125, 0.25
    xi = orc.cheb_nodes(l)
    K = orc.m2l_matrix(l, a, w, t, kernel=K2)
    g = np.array([[m1, m2, m3] for m1 in range(l) for m2 in range(l) for m3 in range(l)])
    x = a * xi[g]                      # target cell centred at 0
    y = w * np.array(t) + a * xi[g]    # source cell centred at w t
    d = x[:, None, :] - y[None, :, :]
    np.testing.assert_allclose(K, 1.0 / (d ** 2).sum(-1), rtol=1e-14)


def test_m2l_homogeneity_degree_minus_two(orc):
    t = (2, -1, 3)
    K1 = orc.m2l_matrix(4, 1.0, 2.0, t, kernel=K2)
    Ka = orc.m2l_matrix(4, 0.0625, 0.125, t, kernel=K2)
    np.testing.assert_allclose(Ka, K1 / 0.0625 ** 2, rtol=1e-13)


def test_fmm_one_and_two_levels_equal_direct(orc):
    pos, q = inputs.uniform_cube(1200, 84)
    pd, fd = orc.direct(pos, q, kernel=K2)
    p1, f1 = orc.Tree(pos, 1).fmm(4, q, kernel=K2)
    assert np.array_equal(p1, pd) and np.array_equal(f1, fd)
    p2, f2 = orc.Tree(pos, 2).fmm(4, q, kernel=K2)
    assert rel(p2, pd) < 1e-14 and rel(f2, fd) < 1e-14


@pytest.mark.parametrize("kind,h,orders", [("cube", 3, range(2, 9)),
                                           ("sphere", 4, range(2, 8))])
def test_fmm_error_falls_with_order(orc, kind, h, orders):
    pos, q = inputs.make(kind, 3000, 85)
    pd, fd = orc.direct(pos, q, kernel=K2)
    t = orc.Tree(pos, h)
    errs = []
    for l in orders:
        p, f = t.fmm(l, q, kernel=K2)
        errs.append(max(rel(p, pd), rel(f, fd)))
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-5, errs


def test_unit_operators_reproduce_exact_m2l(orc):
    # with nothing truncated, the unit-operator path (scaled by a^-2) equals
    # the path that evaluates the kernel at every level
    pos, q = inputs.uniform_cube(3000, 86)
    t = orc.Tree(pos, 4)
    ops, ranks = orc.compressed_unit_ops(3, 0.0, kernel=K2)
    p, f = t.fmm(3, q, kernel=K2)
    pu, fu = t.fmm(3, q, unit_ops=ops, kernel=K2)
    assert rel(pu, p) < 1e-13 and rel(fu, f) < 1e-13
    assert all(r == 27 for r in ranks.values())


def test_kernels_differ_and_bad_kernel_rejected(orc):
    pos, q = inputs.uniform_cube(300, 87)
    p1, _ = orc.direct(pos, q)
    p2, _ = orc.direct(pos, q, kernel=K2)
    assert rel(p1, p2) > 0.1
    with pytest.raises(ValueError):
        orc.direct(pos, q, kernel=3)
    with pytest.raises(ValueError):
        orc.Tree(pos, 3).fmm(3, q, kernel=0)
