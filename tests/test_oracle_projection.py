"""Pins of the projected lattices on the oracle: for a flow that does not vary along z (D2Q9,
nx x ny x 1) or along y and z (D1Q3, nx x 1 x 1), the D3Q19 step maps class sums to class sums.
States with the same class sums F_c (and, for the energy-conserving mode, the same transverse
energies G_c and transverse variance trace) but a different split of each class among its members
step to the same class sums and the same moments.  This is the claim the projected GPU kernels
rest on; the D1Q3 classes of Sec. II B's illustration are the e_x classes.
"""
import numpy as np
import pytest

import oracle
from paper_2501_00620_amd import workloads as wl


def fields(nx, ny, seed, u_max=0.15):
    rho, u, T = wl.fourier_fields(nx, ny, 1, seed=seed, u_max=u_max)
    u = u.copy()
    u[2] = 0.0
    if ny == 1:
        u[1] = 0.0
    return rho, u, T


def stepped_state(nx, ny, mode, seed, steps=3):
    L = oracle.OracleLattice(nx, ny, 1, 0.7, mode=mode)
    L.init(*fields(nx, ny, seed))
    L.step(steps)  # away from equilibrium
    return L


def evolve(L, F, b, steps):
    M = oracle.OracleLattice(L.nx, L.ny, 1, L.tau, mode=["thermal", "iso"][L.mode], T_field=L.T_field)
    M.set_state(F, b)
    M.step(steps)
    return M


def test_classes_partition_the_velocity_set():
    for dims in (2, 1):
        classes, et2 = oracle.projection_classes(dims)
        allidx = np.sort(np.concatenate(classes))
        np.testing.assert_array_equal(allidx, np.arange(19))
        e, w = oracle.velocity_set()
        for c in classes:  # one in-plane member per class, and the class shares its in-plane velocity
            assert (et2[c] == 0).sum() == 1
            assert np.ptp(e[c, 0]) == 0 and (dims == 1 or np.ptp(e[c, 1]) == 0)


@pytest.mark.parametrize("mode", ["thermal", "iso"])
def test_d1q3_split_within_classes_does_not_matter(mode):
    L = stepped_state(12, 1, mode, seed=4)
    F, b = L.state()
    G = F.copy()
    bb = b.copy()
    s = 1e-3 * (1 + 0.5 * np.sin(np.arange(12) * 0.7)).reshape(1, 1, 12)
    # class 0: faces -2s each, edges +s each, rest +4s (sum and sum |e_t|^2 unchanged)
    G[[2, 4, 5, 6]] -= 2 * s
    G[[15, 16, 17, 18]] += s
    G[0] += 4 * s
    # class +1: y faces vs z faces (the transverse energy stays; y-z symmetry is not needed)
    G[[7, 8]] += s
    G[[11, 12]] -= s
    # the transverse variance split between yy and zz
    bb[1] += 0.3 * s[0]
    bb[2] -= 0.3 * s[0]
    Pa = oracle.project(F, b, 1, mode == "thermal")
    Pb = oracle.project(G, bb, 1, mode == "thermal")
    np.testing.assert_allclose(Pa[0], Pb[0], rtol=0, atol=1e-15)
    A, B = evolve(L, F, b, 20), evolve(L, G, bb, 20)
    for x, y in zip(oracle.project(A.F, A.b, 1, mode == "thermal"), oracle.project(B.F, B.b, 1, mode == "thermal")):
        np.testing.assert_allclose(x, y, rtol=0, atol=1e-14)
    for x, y in zip(A.moments(), B.moments()):
        np.testing.assert_allclose(x, y, rtol=0, atol=1e-14)
    # one step on, the populations themselves still differ (the test above is not vacuous; the
    # difference within classes relaxes as (1 - omega)^t)
    A1, B1 = evolve(L, F, b, 1), evolve(L, G, bb, 1)
    assert np.abs(A1.F - B1.F).max() > 1e-5
    for x, y in zip(oracle.project(A1.F, A1.b, 1, mode == "thermal"), oracle.project(B1.F, B1.b, 1, mode == "thermal")):
        np.testing.assert_allclose(x, y, rtol=0, atol=1e-15)


def test_iso_ignores_the_transverse_energy_and_variance():
    # ISO keeps no G and no transverse variance: moving mass between a class's in-plane and
    # transverse members, and changing bbar_zz, leave the in-plane evolution unchanged
    L = stepped_state(9, 7, "iso", seed=8)
    F, b = L.state()
    G = F.copy()
    bb = b.copy()
    s = 2e-3
    for i_in, pair in ((0, (5, 6)), (1, (11, 12)), (3, (13, 14)), (2, (15, 16)), (4, (17, 18))):
        G[i_in] -= s
        G[list(pair)] += s / 2
    bb[2] += 0.01
    A, B = evolve(L, F, b, 15), evolve(L, G, bb, 15)
    for x, y in zip(oracle.project(A.F, A.b, 2, False), oracle.project(B.F, B.b, 2, False)):
        np.testing.assert_allclose(x, y, rtol=0, atol=1e-14)
    ra, ua, _ = A.moments()
    rb, ub, _ = B.moments()
    np.testing.assert_allclose(ra, rb, rtol=0, atol=1e-14)
    np.testing.assert_allclose(ua, ub, rtol=0, atol=1e-14)


@pytest.mark.parametrize("dims,shape", [(2, (9, 7)), (1, (12, 1))])
def test_transverse_velocity_and_variance_stay_zero(dims, shape):
    L = stepped_state(shape[0], shape[1], "thermal", seed=5, steps=10)
    _, u, _ = L.moments()
    assert np.abs(u[2]).max() < 1e-15
    assert np.abs(L.b[4]).max() < 1e-15 and np.abs(L.b[5]).max() < 1e-15
    if dims == 1:
        assert np.abs(u[1]).max() < 1e-15 and np.abs(L.b[3]).max() < 1e-15
