"""Pins of the oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: moment
identities of the lattice, the textbook BGK collision, stated invariants,
special cases, closed forms, brute force and the printed parameter tables.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import mc_inputs
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


LATTICES = pytest.mark.parametrize("q", [27, 19])


def random_state(seed, n, amp_u=0.05, amp_noise=1e-3, rho_noise=1e-3, q=27):
    """Non-equilibrium populations: equilibrium of a random (rho, u) field plus noise."""
    rng = np.random.default_rng(seed)
    ncell = n ** 3
    rho = 1.0 + rng.uniform(-rho_noise, rho_noise, ncell)
    u = rng.uniform(-amp_u, amp_u, (ncell, 3))
    c, w = oracle.velocity_set(q)
    cu = u @ c.T
    usq = np.sum(u * u, axis=1)[:, None]
    f = rho[:, None] * w[None, :] * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * usq)
    f *= 1.0 + rng.uniform(-amp_noise, amp_noise, f.shape)
    return np.ascontiguousarray(f)


WCLASS = {27: {0: 8 / 27, 1: 2 / 27, 2: 1 / 54, 3: 1 / 216},   # D3Q27
          19: {0: 1 / 3, 1: 1 / 18, 2: 1 / 36}}                # D3Q19 (no corners)


def lattice_velocities(q):
    """The velocities in index order: {-1,0,1}^3 with cx slowest; D3Q19 leaves
    out the eight corners."""
    return [v for v in itertools.product((-1, 0, 1), repeat=3) if q == 27 or np.count_nonzero(v) < 3]


def textbook_feq(rho, u, q=27):
    """Second-order Maxwellian truncation written from the textbook form with
    c_s^2 = 1/3 and the textbook weights by number of non-zero velocity
    components."""
    vel = lattice_velocities(q)
    out = np.zeros(q)
    for i, v in enumerate(vel):
        cvec = np.array(v, float)
        w = WCLASS[q][int(np.count_nonzero(cvec))]
        cu = cvec @ u
        out[i] = rho * w * (1 + cu / (1 / 3) + (cu ** 2 - np.dot(u, u) / 3) / (2 / 9))
    return out


# ---------------------------------------------------------------- lattice
def test_velocity_set_index_convention_and_weights():
    c, w = oracle.velocity_set()
    for i, (cx, cy, cz) in enumerate(itertools.product((-1, 0, 1), repeat=3)):
        assert tuple(c[i]) == (cx, cy, cz)
        assert tuple(c[26 - i]) == (-cx, -cy, -cz)
    # the weights are fixed by the isotropy conditions of a 27-velocity set
    # with symmetric classes: sum w = 1, sum w cx^2 = 1/3, sum w cx^2 cy^2 = 1/9,
    # sum w cx^2 cy^2 cz^2 = 1/27
    cf = c.astype(float)
    assert abs(w.sum() - 1) < 1e-15
    assert abs(np.sum(w * cf[:, 0] ** 2) - 1 / 3) < 1e-15
    assert abs(np.sum(w * cf[:, 0] ** 2 * cf[:, 1] ** 2) - 1 / 9) < 1e-15
    assert abs(np.sum(w * cf[:, 0] ** 2 * cf[:, 1] ** 2 * cf[:, 2] ** 2) - 1 / 27) < 1e-15
    # isotropy through fourth order
    for a, b in itertools.product(range(3), repeat=2):
        assert abs(np.sum(w * cf[:, a] * cf[:, b]) - (a == b) / 3) < 1e-15
    for a, b, g, d in itertools.product(range(3), repeat=4):
        iso = ((a == b) * (g == d) + (a == g) * (b == d) + (a == d) * (b == g)) / 9
        assert abs(np.sum(w * cf[:, a] * cf[:, b] * cf[:, g] * cf[:, d]) - iso) < 1e-15
    for a, b, g in itertools.product(range(3), repeat=3):
        assert abs(np.sum(w * cf[:, a] * cf[:, b] * cf[:, g])) < 1e-15


def test_d3q19_velocity_set_and_weights():
    """D3Q19: the D3Q27 order without corners, opposite q-1-i, and weights
    fixed by sum w = 1, sum w cx^2 = 1/3, sum w cx^2 cy^2 = 1/9 (three
    classes, three conditions); isotropic through fourth order."""
    c, w = oracle.velocity_set(19)
    vel = lattice_velocities(19)
    assert len(vel) == 19
    for i in range(19):
        assert tuple(c[i]) == vel[i]
        assert tuple(c[18 - i]) == tuple(-np.array(vel[i]))
    cf = c.astype(float)
    nz = np.count_nonzero(c, axis=1)
    A = np.array([[1, 6, 12], [0, 2, 8], [0, 0, 4]], float)   # the three conditions per class
    wc = np.linalg.solve(A, [1, 1 / 3, 1 / 9])
    assert np.max(np.abs(w - wc[nz])) < 1e-15
    for a, b in itertools.product(range(3), repeat=2):
        assert abs(np.sum(w * cf[:, a] * cf[:, b]) - (a == b) / 3) < 1e-15
    for a, b, g, d in itertools.product(range(3), repeat=4):
        iso = ((a == b) * (g == d) + (a == g) * (b == d) + (a == d) * (b == g)) / 9
        assert abs(np.sum(w * cf[:, a] * cf[:, b] * cf[:, g] * cf[:, d]) - iso) < 1e-15
    for a, b, g in itertools.product(range(3), repeat=3):
        assert abs(np.sum(w * cf[:, a] * cf[:, b] * cf[:, g])) < 1e-15


@pytest.mark.parametrize("q,groups", [(27, [4, 5, 18]), (19, [4, 5, 10])])
def test_moment_basis_invertible_and_grouped(q, groups):
    """Table 1's groups: kinematic (4), shear (5), hom (T, and Q and A: the
    raw moments of order >= 3 that the lattice supports)."""
    M, Minv, g = oracle.moment_basis(q)
    assert np.max(np.abs(M @ Minv - np.eye(q))) < 1e-13
    assert list(np.bincount(g)) == groups
    assert np.linalg.matrix_rank(M) == q


@LATTICES
def test_equilibrium_moments(q):
    """The truncated Maxwellian reproduces rho, rho u and rho/3 I + rho u u."""
    c, _ = oracle.velocity_set(q)
    cf = c.astype(float)
    rng = np.random.default_rng(1)
    for _ in range(10):
        rho = 1 + rng.uniform(-0.1, 0.1)
        u = rng.uniform(-0.1, 0.1, 3)
        feq = oracle.equilibrium(rho, u, q)
        assert np.max(np.abs(feq - textbook_feq(rho, u, q))) < 1e-16
        assert abs(feq.sum() - rho) < 1e-15
        assert np.max(np.abs(cf.T @ feq - rho * u)) < 1e-16
        P = (cf.T * feq) @ cf
        assert np.max(np.abs(P - (rho / 3 * np.eye(3) + rho * np.outer(u, u)))) < 1e-15


# ---------------------------------------------------------------- collision pins
@LATTICES
def test_equilibrium_is_fixed_point(q):
    rng = np.random.default_rng(2)
    for omega in (0.7, 1.3, 1.99):
        for _ in range(5):
            feq = oracle.equilibrium(1 + rng.uniform(-0.05, 0.05), rng.uniform(-0.08, 0.08, 3), q)
            fs, gamma, ds, dh = oracle.collide(feq, omega)
            assert np.max(np.abs(fs - feq)) < 5e-16
            assert np.max(np.abs(ds)) < 5e-16 and np.max(np.abs(dh)) < 5e-16


@LATTICES
def test_uniform_state_stays_bitwise_uniform(q):
    n = 6
    feq = oracle.equilibrium(1.01, np.array([0.03, -0.02, 0.01]), q)
    f = np.ascontiguousarray(np.tile(feq, (n ** 3, 1)))
    oracle.run(f, n, 3, 1.9)
    assert np.all(f == f[0:1, :])
    assert np.max(np.abs(f[0] - feq)) < 5e-16


@LATTICES
def test_collision_conserves_mass_and_momentum(q):
    c, _ = oracle.velocity_set(q)
    cf = c.astype(float)
    f = random_state(3, 3, amp_noise=5e-2, q=q)
    for omega in (0.5, 1.0, 1.5, 1.999):
        for cell in range(f.shape[0]):
            fs, *_ = oracle.collide(f[cell], omega)
            assert abs(fs.sum() - f[cell].sum()) < 1e-15
            assert np.max(np.abs(cf.T @ (fs - f[cell]))) < 1e-15


@LATTICES
def test_step_conserves_totals(q):
    n = 8
    c, _ = oracle.velocity_set(q)
    f = random_state(4, n, amp_noise=1e-2, q=q)
    mass0 = f.sum()
    j0 = (f @ c.astype(float)).sum(axis=0)
    oracle.run(f, n, 5, 1.95)
    assert abs(f.sum() - mass0) / mass0 < 1e-14
    assert np.max(np.abs((f @ c.astype(float)).sum(axis=0) - j0)) < 1e-14 * mass0


@LATTICES
def test_bgk_special_cases(q):
    """gamma = 2 gives the textbook BGK collision; at omega = 1 the closed-form
    gamma is exactly 2, so KBC collapses to BGK with f* = f^eq."""
    f = random_state(5, 2, amp_noise=2e-2, q=q)
    c, _ = oracle.velocity_set(q)
    for cell in range(f.shape[0]):
        rho = f[cell].sum()
        u = (c.astype(float).T @ f[cell]) / rho
        feq = textbook_feq(rho, u, q)
        for omega in (0.8, 1.6, 1.97):
            fs, gamma, *_ = oracle.collide(f[cell], omega, oracle.MODE_BGK)
            assert gamma == 2.0
            assert np.max(np.abs(fs - (f[cell] - omega * (f[cell] - feq)))) < 1e-15
        fs, gamma, *_ = oracle.collide(f[cell], 1.0)
        assert abs(gamma - 2.0) < 1e-14
        assert np.max(np.abs(fs - feq)) < 1e-15


@LATTICES
def test_shear_hom_split(q):
    """ds carries exactly the traceless and off-diagonal second moments of
    f^neq and no other raw moment; ds + dh = f^neq; closed form of ds (the
    same class-wise formulas on both lattices: corners carry no shear part)."""
    c, w = oracle.velocity_set(q)
    cf = c.astype(float)
    f = random_state(6, 2, amp_noise=3e-2, q=q)
    for cell in range(f.shape[0]):
        fc = f[cell]
        rho = fc.sum()
        u = (cf.T @ fc) / rho
        fneq = fc - textbook_feq(rho, u, q)
        _, _, ds, dh = oracle.collide(fc, 1.7)
        assert np.max(np.abs(ds + dh - fneq)) < 1e-15

        def mom(v, a, b, e):
            return np.sum(v * cf[:, 0] ** a * cf[:, 1] ** b * cf[:, 2] ** e)

        nxz = mom(fneq, 2, 0, 0) - mom(fneq, 0, 0, 2)
        nyz = mom(fneq, 0, 2, 0) - mom(fneq, 0, 0, 2)
        assert abs(mom(ds, 2, 0, 0) - mom(ds, 0, 0, 2) - nxz) < 1e-16
        assert abs(mom(ds, 0, 2, 0) - mom(ds, 0, 0, 2) - nyz) < 1e-16
        for (a, b, e) in ((1, 1, 0), (1, 0, 1), (0, 1, 1)):
            assert abs(mom(ds, a, b, e) - mom(fneq, a, b, e)) < 1e-16
        assert abs(mom(ds, 2, 0, 0) + mom(ds, 0, 2, 0) + mom(ds, 0, 0, 2)) < 1e-16
        for a, b, e in itertools.product(range(3), repeat=3):
            if a + b + e <= 1 or a + b + e >= 3:
                assert abs(mom(ds, a, b, e)) < 1e-16
        # closed form per velocity class
        exp = np.zeros(q)
        pxy, pxz, pyz = mom(fneq, 1, 1, 0), mom(fneq, 1, 0, 1), mom(fneq, 0, 1, 1)
        for i in range(q):
            cx, cy, cz = c[i]
            nz = np.count_nonzero(c[i])
            if nz == 1:
                exp[i] = ((2 * nxz - nyz) / 6 if cx else (2 * nyz - nxz) / 6 if cy else -(nxz + nyz) / 6)
            elif nz == 2:
                exp[i] = (cx * cy * pxy + cx * cz * pxz + cy * cz * pyz) / 4
        assert np.max(np.abs(exp - ds)) < 1e-16


@LATTICES
def test_closed_form_gamma_minimises_quadratic_entropy(q):
    """The closed form makes the quadratic expansion of H around f^eq,
    sum (f* - f^eq)^2 / f^eq, stationary in gamma."""
    c, _ = oracle.velocity_set(q)
    f = random_state(7, 2, amp_noise=2e-2, q=q)
    for cell in range(f.shape[0]):
        fc = f[cell]
        rho = fc.sum()
        u = (c.astype(float).T @ fc) / rho
        feq = textbook_feq(rho, u, q)
        omega = 1.93
        _, gamma, ds, dh = oracle.collide(fc, omega)

        def hq(g):
            fs = fc - omega * ds - omega * g / 2 * dh
            return np.sum((fs - feq) ** 2 / feq)

        d = 1e-3 * max(1.0, abs(gamma))
        assert hq(gamma) <= hq(gamma + d) and hq(gamma) <= hq(gamma - d)
        slope = (hq(gamma + d) - hq(gamma - d)) / (2 * d)
        curv = (hq(gamma + d) - 2 * hq(gamma) + hq(gamma - d)) / d ** 2
        assert abs(slope) < 1e-6 * curv * d + 1e-30


@LATTICES
def test_exact_entropic_gamma_limit(q):
    """Near equilibrium and at rest the closed form approaches the exact
    minimiser of the discrete H-function, and the exact minimiser never
    increases H."""
    rng = np.random.default_rng(8)
    c, w = oracle.velocity_set(q)
    omega = 1.98
    diffs = []
    for amp in (1e-2, 1e-3, 1e-4):
        dd = []
        for _ in range(10):
            feq = oracle.equilibrium(1.0, np.zeros(3), q)
            f = feq * (1 + amp * rng.uniform(-1, 1, q))
            # restore the mass and momentum of the rest state so that u = 0
            f = f - w * (f.sum() - 1.0)
            jx = c.astype(float).T @ f
            for a in range(3):
                sel_p = c[:, a] == 1
                sel_m = c[:, a] == -1
                f[sel_p] -= jx[a] / 2 * w[sel_p] / w[sel_p].sum()
                f[sel_m] += jx[a] / 2 * w[sel_m] / w[sel_m].sum()
            assert np.max(np.abs(c.astype(float).T @ f)) < 1e-15
            _, g_cf, _, _ = oracle.collide(f, omega, oracle.MODE_KBC)
            fs_ex, g_ex, _, _ = oracle.collide(f, omega, oracle.MODE_EXACT)
            H = lambda v: np.sum(v * np.log(v / w))
            assert H(fs_ex) <= H(f) + 1e-15
            dd.append(abs(g_cf - g_ex))
        diffs.append(np.median(dd))
    assert diffs[1] < diffs[0] / 2 and diffs[2] < diffs[1] / 2
    assert diffs[2] < diffs[0] / 20 and diffs[2] < 1e-5


@pytest.mark.slow
def test_gamma_approaches_bgk_value_under_refinement():
    """For a resolved flow the mean stabiliser tends to the BGK value 2 as the
    resolution grows (remark on the convergence of the deterministic scheme)."""
    dev = []
    for n in (16, 32):
        u0 = 0.05 * 32 / n
        omega = oracle.omega_shear(oracle.lattice_viscosity(n, u0, 100.0))
        f = oracle.init_populations(n, u0, 0.0, np.zeros(24), False)
        gs = oracle.run(f, n, 20 * (n // 16) ** 2, omega, gamma_stats=True)
        dev.append(abs(gs[-1, 2] - 2.0))
    assert dev[1] < dev[0] / 3


# ---------------------------------------------------------------- lattice symmetry
def _cube_symmetries():
    mats = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            R = np.zeros((3, 3), int)
            for r in range(3):
                R[r, perm[r]] = signs[r]
            mats.append(R)
    return mats


def _apply_symmetry(f, n, R):
    q = f.shape[1]
    c, _ = oracle.velocity_set(q)
    sigma = np.zeros(q, int)
    for i in range(q):
        rc = R @ c[i]
        sigma[i] = [k for k in range(q) if tuple(c[k]) == tuple(rc)][0]
    fz = f.reshape(n, n, n, q)
    out = np.zeros_like(fz)
    idx = np.arange(n)
    Z, Yg, X = np.meshgrid(idx, idx, idx, indexing="ij")
    P = np.stack([X, Yg, Z], axis=-1)
    Pn = np.einsum("ab,zyxb->zyxa", R, P) % n
    for i in range(q):
        out[Pn[..., 2], Pn[..., 1], Pn[..., 0], sigma[i]] = fz[..., i]
    return np.ascontiguousarray(out.reshape(n ** 3, q))


@LATTICES
def test_cube_symmetry_equivariance(q):
    n = 6
    f0 = random_state(9, n, amp_noise=5e-3, q=q)
    rng = np.random.default_rng(10)
    syms = _cube_symmetries()
    assert len(syms) == 48
    for k in rng.choice(48, size=6, replace=False):
        R = syms[k]
        a = f0.copy()
        b = _apply_symmetry(f0, n, R)
        oracle.run(a, n, 3, 1.97)
        oracle.run(b, n, 3, 1.97)
        assert np.max(np.abs(_apply_symmetry(a, n, R) - b)) < 1e-15


# ---------------------------------------------------------------- streaming
@LATTICES
def test_streaming_is_a_permutation_and_keeps_relative_entropy(q):
    n = 6
    c, w = oracle.velocity_set(q)
    f = random_state(11, n, amp_noise=1e-2, q=q)
    g = f.copy()
    oracle.run(g, n, 1, 0.0, mode=oracle.MODE_BGK)   # zero frequency: streaming only
    for i in range(q):
        assert np.array_equal(np.sort(f[:, i]), np.sort(g[:, i]))
    # single-velocity shift check
    fz = f.reshape(n, n, n, q)
    gz = g.reshape(n, n, n, q)
    for i in range(q):
        cx, cy, cz = c[i]
        assert np.array_equal(gz[..., i], np.roll(fz[..., i], shift=(cz, cy, cx), axis=(0, 1, 2)))
    hrel = lambda v: np.sum(v * np.log(v / w) - v + w)
    assert abs(hrel(f) - hrel(g)) <= 1e-12 * hrel(f)


def test_initial_relative_entropy_scales_with_dx_squared():
    """Lemma (well-prepared initialisation): H_rel(0) = O(eps^2) when the lattice
    velocity shrinks with eps (diffusive scaling)."""
    _, w = oracle.velocity_set()
    y = mc_inputs.draw_y(5, 1)[0]
    vals = []
    for n in (8, 16, 32):
        eps = 2 * math.pi / n
        f = oracle.init_populations(n, 0.05 * 8 / n, 0.05, y, True)
        vals.append(eps ** 3 * np.sum(f * np.log(f / w) - f + w))
    r1, r2 = vals[0] / vals[1], vals[1] / vals[2]
    assert 3.8 < r1 < 4.2 and 3.9 < r2 < 4.1


# ---------------------------------------------------------------- initial data
@LATTICES
def test_initial_kinetic_energy_closed_form(q):
    """Discrete orthogonality: KE(0) = U0^2 (1/8 + amp^2 sum Y^2 / 1024)
    without projection."""
    for n, seed in ((8, 1), (12, 2), (16, 3)):
        y = mc_inputs.draw_y(seed, 1)[0]
        u0, amp = 0.05, 0.3
        f = oracle.init_populations(n, u0, amp, y, False, q)
        rho, u = oracle.moments(f, n)
        ke = oracle.kinetic_energy(u)
        assert abs(ke - u0 ** 2 * (1 / 8 + amp ** 2 * np.sum(y ** 2) / 1024)) < 1e-15
        assert np.max(np.abs(rho - 1)) < 1e-15


@LATTICES
def test_initial_populations_carry_the_prescribed_velocity(q):
    """eq. (initialPopulations): the populations of a node are the equilibrium
    of density 1 and the node's velocity, so their zeroth moment is 1 and their
    first moment is that velocity, component by component (moments taken here
    from the listed velocities, not from the oracle)."""
    n = 6
    rng = np.random.default_rng(21)
    u = rng.uniform(-0.08, 0.08, (3, n, n, n))
    u[1] *= 0.5     # distinct scales per component
    u[2] *= 0.25
    y = mc_inputs.draw_y(22, 1)[0]
    cf = np.array(lattice_velocities(q), dtype=float)
    cases = ((oracle.equilibrium_field(u, q), u),
             (oracle.init_populations(n, 0.04, 0.3, y, True, q), oracle.initial_velocity(n, 0.04, 0.3, y, True)))
    for f, target in cases:
        assert f.shape == (n ** 3, q)
        assert np.max(np.abs(f.sum(axis=1) - 1.0)) < 1e-15
        j = f @ cf
        for a in range(3):
            assert np.max(np.abs(j[:, a] - target[a].ravel())) < 1e-16


@LATTICES
def test_moments_of_equilibrium_states_and_uniform_flow_reductions(q):
    """Density and velocity are the zeroth moment and the first moment over
    the zeroth: the moments of equilibrium populations f^eq(rho, u), built
    here from the textbook form, return rho and u at every node. A uniform
    flow of velocity U at density 1 on N^3 nodes has mass N^3, momentum
    N^3 U and kinetic energy |U|^2 / 2."""
    n = 3
    rng = np.random.default_rng(23)
    rho = 1.0 + rng.uniform(-0.05, 0.05, n ** 3)
    u = rng.uniform(-0.08, 0.08, (n ** 3, 3))
    f = np.stack([textbook_feq(rho[k], u[k], q) for k in range(n ** 3)])
    r, v = oracle.moments(f, n)
    assert np.max(np.abs(r.ravel() - rho)) < 1e-15
    for a in range(3):
        assert np.max(np.abs(v[a].ravel() - u[:, a])) < 1e-15
    U = np.array([0.03, -0.02, 0.01])
    f = np.tile(textbook_feq(1.0, U, q), (n ** 3, 1))
    red = oracle.reductions(f, n)
    exp = [n ** 3, n ** 3 * U[0], n ** 3 * U[1], n ** 3 * U[2], 0.5 * np.dot(U, U)]
    assert np.max(np.abs(red - exp)) < 1e-14


def test_leray_projection_properties():
    """The projection is idempotent, leaves a spectrally divergence-free field,
    removes a pure gradient, has rank 16 on the 24 perturbation fields, and
    matches the closed form s + grad(div s)/12 (all fields are Laplacian
    eigenfunctions with eigenvalue -12)."""
    n = 8
    X, Y, Z = oracle.grid(n)
    k = np.fft.fftfreq(n) * n
    KZ, KY, KX = np.meshgrid(k, k, k, indexing="ij")
    cols = []
    for p in range(24):
        e = np.zeros(24)
        e[p] = 1
        s = oracle.perturbation(n, e)
        ps = oracle.leray_project(s)
        assert np.max(np.abs(oracle.leray_project(ps) - ps)) < 1e-14
        div = KX * np.fft.fftn(ps[0]) + KY * np.fft.fftn(ps[1]) + KZ * np.fft.fftn(ps[2])
        assert np.max(np.abs(div)) < 1e-11
        # residual is curl-free
        r = [np.fft.fftn(s[a] - ps[a]) for a in range(3)]
        curl = (KY * r[2] - KZ * r[1], KZ * r[0] - KX * r[2], KX * r[1] - KY * r[0])
        assert max(np.max(np.abs(cc)) for cc in curl) < 1e-11
        # closed form by analytic derivatives
        al, i, j, kk = p // 8, (p // 4) % 2, (p // 2) % 2, p % 2
        fn = (np.sin, np.cos)
        dfn = (lambda t: 2 * np.cos(t), lambda t: -2 * np.sin(t))
        d2fn = (lambda t: -4 * np.sin(t), lambda t: -4 * np.cos(t))
        idxs = (i, j, kk)
        coords = (2 * X, 2 * Y, 2 * Z)
        grad_div = np.zeros((3, n, n, n))
        for b in range(3):
            term = np.ones((n, n, n)) / 8
            for ax in range(3):
                if ax == al and ax == b:
                    term = term * d2fn[idxs[ax]](coords[ax])
                elif ax == al or ax == b:
                    term = term * dfn[idxs[ax]](coords[ax])
                else:
                    term = term * fn[idxs[ax]](coords[ax])
            grad_div[b] = term
        assert np.max(np.abs(ps - (s + grad_div / 12))) < 1e-14
        cols.append(ps.ravel())
    assert np.linalg.matrix_rank(np.array(cols), tol=1e-9) == 16


# ---------------------------------------------------------------- analytic decay
@pytest.mark.slow
@LATTICES
def test_two_dimensional_taylor_green_decay_rate(q):
    """A z-independent 2-D Taylor-Green mode decays like exp(-2 nu k^2 t), so
    its kinetic energy like exp(-4 nu k^2 t), k = 2 pi / n per lattice unit."""
    n = 24
    u0 = 0.01
    nu = 0.05
    omega = oracle.omega_shear(nu)
    X, Y, Z = oracle.grid(n)
    u = u0 * np.stack([np.sin(X) * np.cos(Y), -np.cos(X) * np.sin(Y), np.zeros_like(X)])
    f = oracle.equilibrium_field(u, q)
    steps = 120
    oracle.run(f, n, 20, omega)      # let the initial pressure transient pass
    _, ua = oracle.moments(f, n)
    ke_a = oracle.kinetic_energy(ua)
    oracle.run(f, n, steps, omega)
    _, ub = oracle.moments(f, n)
    ke_b = oracle.kinetic_energy(ub)
    rate = -math.log(ke_b / ke_a) / steps
    k = 2 * math.pi / n
    assert abs(rate / (4 * nu * k ** 2) - 1) < 0.01


# ---------------------------------------------------------------- parameter tables
def test_unit_conversion_reproduces_paper_tables():
    with open(os.path.join(GOLDEN, "paper_parameter_tables.json")) as fh:
        tab = json.load(fh)
    for row in tab["rows"]:
        n = row["N"]
        dx = 2 * math.pi / (n - 1) if row["dx"] == "2pi/(N-1)" else 2 * math.pi / n
        tau, dt = oracle.paper_table_row(n, row["Ma"], row["Re"], dx)
        assert round(tau, 6) == pytest.approx(row["tau"], abs=0), row
        mant, ex = row["dt"]
        # three printed digits: within one unit of the last one
        assert abs(dt / 10 ** ex - mant) < 0.01, row


def test_lattice_viscosity_reproduces_table_rows_with_dx_2pi_over_n():
    """Re = U l / nu with l = 1 on the periodic box of side 2 pi: with dx =
    2 pi / N a unit length is N / (2 pi) lattice units. The rows of Table 3
    printed with that spacing (N >= 32) give their tau back from the lattice
    viscosity, at the lattice velocity Ma c_s."""
    with open(os.path.join(GOLDEN, "paper_parameter_tables.json")) as fh:
        rows = [r for r in json.load(fh)["rows"] if r["dx"] == "2pi/N"]
    assert len(rows) == 5
    for row in rows:
        nu = oracle.lattice_viscosity(row["N"], row["Ma"] * math.sqrt(1.0 / 3.0), row["Re"])
        tau = 1.0 / oracle.omega_shear(nu)
        assert abs(tau - (3.0 * nu + 0.5)) < 1e-15
        assert round(tau, 6) == pytest.approx(row["tau"], abs=0), row


# ---------------------------------------------------------------- complex step
@LATTICES
def test_complex_step_matches_central_differences(q):
    n, steps = 8, 6
    y = mc_inputs.draw_y(3, 1)[0]
    g = oracle.ke_gradient_complex_step(n, 0.05, 100.0, 0.5, y, True, steps, params=[0, 5, 13, 23], q=q)
    h = 1e-4
    for p in (0, 5, 13, 23):
        yp, ym = y.copy(), y.copy()
        yp[p] += h
        ym[p] -= h
        fd = (oracle.ke_after(n, 0.05, 100.0, 0.5, yp, True, steps, q=q) -
              oracle.ke_after(n, 0.05, 100.0, 0.5, ym, True, steps, q=q)) / (2 * h)
        assert abs(fd - g[p]) <= 1e-6 * abs(g).max() + 1e-14


@LATTICES
def test_complex_step_through_the_exact_stabiliser(q):
    """The exact stabiliser in complex arithmetic (the real minimiser by
    bisection, then Newton steps on dH/dt = 0 in complex numbers) gives the
    derivative of the collision: its complex step equals the central
    differences of the real bisection-only collision, which converge to it
    like the square of the difference step. Then the same through a few
    steps of a small lattice."""
    rng = np.random.default_rng(31)
    _, w = oracle.velocity_set(q)
    h = 1e-30
    for _ in range(4):
        u = rng.uniform(-0.06, 0.06, 3)
        f = oracle.equilibrium(1.0 + rng.uniform(-0.02, 0.02), u, q) * (1 + rng.uniform(-3e-2, 3e-2, q))
        v = rng.normal(size=q)
        om = rng.uniform(1.5, 1.99)
        fz, gz = oracle.collide_complex(f + 1j * h * v, om, oracle.MODE_EXACT)
        fr, gr, *_ = oracle.collide(f, om, oracle.MODE_EXACT)
        assert np.max(np.abs(fz.real - fr)) < 1e-16 and abs(gz.real - gr) < 1e-13
        errs = []
        for eps in (1e-5, 1e-6, 1e-7):
            fp, gp, *_ = oracle.collide(f + eps * v, om, oracle.MODE_EXACT)
            fm, gm, *_ = oracle.collide(f - eps * v, om, oracle.MODE_EXACT)
            errs.append(max(abs(gz.imag / h - (gp - gm) / (2 * eps)) / abs(gz.imag / h),
                            np.max(np.abs(fz.imag / h - (fp - fm) / (2 * eps))) / np.max(np.abs(fz.imag / h))))
        assert errs[1] < 1e-3 and errs[2] < 1e-5, errs
        assert errs[0] > 50 * errs[1], errs      # second order in the difference step
    n, steps = 8, 4
    y = mc_inputs.draw_y(4, 1)[0]
    args = (n, 0.05, 100.0, 0.5)
    g = oracle.ke_gradient_complex_step(*args, y, True, steps, params=[2, 17], q=q, mode=oracle.MODE_EXACT)
    gk = oracle.ke_gradient_complex_step(*args, y, True, steps, params=[2, 17], q=q)
    dh = 1e-4
    for p in (2, 17):
        yp, ym = y.copy(), y.copy()
        yp[p] += dh
        ym[p] -= dh
        fd = (oracle.ke_after(*args, yp, True, steps, q=q, mode=oracle.MODE_EXACT) -
              oracle.ke_after(*args, ym, True, steps, q=q, mode=oracle.MODE_EXACT)) / (2 * dh)
        assert abs(fd - g[p]) <= 1e-6 * abs(g).max() + 1e-14
    assert np.max(np.abs(g - gk)) > 0.0   # the stabiliser differs from the closed form


def test_exact_stabiliser_change_does_not_vanish_near_equilibrium():
    """With the second-order equilibrium, ln(f^eq_i / w_i) = 3 c_i.u - 1.5 |u|^2
    + O(u^3) (the quadratic terms cancel), and dh has no mass or momentum, so
    the root of sum_i dh_i ln(f*_i / w_i) sits where t dh balances the
    third-order part: along f = f^eq + eps d (d in the hom group) the exact
    minimiser moves f* away from the closed form by an amount independent of
    eps, and gamma grows like 1/eps. Its derivative therefore grows without
    bound near equilibrium."""
    rng = np.random.default_rng(3)
    M, Minv, grp = oracle.moment_basis(27)
    u = np.array([0.04, -0.03, 0.02])
    feq = oracle.equilibrium(1.0, u, 27)
    m = M @ rng.normal(size=27)
    m[grp != 2] = 0.0
    d = Minv @ m
    gaps, gammas = [], []
    for eps in (1e-5, 1e-7, 1e-9, 1e-11):
        fe, ge, *_ = oracle.collide(feq + eps * d, 1.9, oracle.MODE_EXACT)
        fk, _, *_ = oracle.collide(feq + eps * d, 1.9, oracle.MODE_KBC)
        gaps.append(np.max(np.abs(fe - fk)))
        gammas.append(ge * eps)
    assert 1e-7 < gaps[0] < 1e-4   # third order in u ~ 0.04
    assert max(gaps) / min(gaps) < 1.01
    assert abs(gammas[3] / gammas[2] - 1) < 1e-2   # gamma ~ 1/eps once it dominates the O(1) part


# ---------------------------------------------------------------- observables
def test_spectrum_of_taylor_green_sits_in_shell_two():
    n = 16
    u = oracle.taylor_green(n)
    E = oracle.energy_spectrum(u)
    # the 8 wave vectors (+-1, +-1, +-1) have |k| = sqrt 3 -> shell 2;
    # shell 2 holds |k|^2 in {3, 4, 5, 6}: 8 + 6 + 24 + 24 = 62 modes
    phi_total = 2 * oracle.kinetic_energy(u)
    assert abs(E[2] - 4 * math.pi / 62 * 0.5 * 3 * phi_total) < 1e-14
    assert np.max(np.abs(np.delete(E, 2))) < 1e-14


def test_structure_function_matches_direct_sum():
    n = 8
    rng = np.random.default_rng(12)
    u = rng.normal(size=(3, n, n, n))
    S = oracle.structure_function(u)
    # direct O(N^6) evaluation of the shell-averaged squared increment
    h = np.arange(n)
    hm = np.where(h > n // 2, h - n, h)
    acc = np.zeros(n // 2)
    cnt = np.zeros(n // 2)
    for hz in range(n):
        for hy in range(n):
            for hx in range(n):
                r = int(math.floor(math.sqrt(hm[hx] ** 2 + hm[hy] ** 2 + hm[hz] ** 2) + 0.5))
                if 1 <= r <= n // 2:
                    sh = np.roll(u, shift=(-hz, -hy, -hx), axis=(1, 2, 3))
                    acc[r - 1] += np.mean(np.sum((sh - u) ** 2, axis=0))
                    cnt[r - 1] += 1
    assert np.max(np.abs(S - acc / cnt)) < 1e-12


def test_wasserstein_sorted_matches_permutation_brute_force():
    rng = np.random.default_rng(13)
    for m in range(1, 8):
        a = rng.normal(size=m)
        b = rng.normal(size=m) + 0.3
        brute = min(np.mean(np.abs(a - b[list(p)])) for p in itertools.permutations(range(m)))
        assert abs(oracle.wasserstein1_equal_weights(a, b) - brute) < 1e-15


def test_sample_error_closed_forms():
    """eq. (sample_error): zero for identical ensembles; |delta_m| averaged
    over samples (not pooled over them) when a = (1 + delta_m) b; the
    reference in the denominator; the absolute value; the Euclidean length
    for the vector (a 3-4-5 reference); 0/0 where a reference component
    vanishes."""
    rng = np.random.default_rng(21)
    b = rng.normal(size=(2, 3, 8))
    assert np.array_equal(oracle.sample_error_l1(b, b), np.zeros(4))
    b[1] *= 1e3
    a = b * np.array([1.1, 1.3])[:, None, None]
    assert np.max(np.abs(oracle.sample_error_l1(a, b) - 0.2)) < 1e-15
    assert np.max(np.abs(oracle.sample_error_l1(-b, b) - 2.0)) < 1e-15
    one = np.ones((1, 3, 8))
    assert np.max(np.abs(oracle.sample_error_l1(one, 0.5 * one) - 1.0)) < 1e-15
    assert np.max(np.abs(oracle.sample_error_l1(0.5 * one, one) - 0.5)) < 1e-15
    ref = np.zeros((1, 3, 8))
    ref[0, 0], ref[0, 1] = 3.0, 4.0
    got = oracle.sample_error_l1(ref + np.array([0.01, 0.0, 0.0])[None, :, None], ref)
    assert abs(got[0] - 0.01 / 3) < 1e-15 and got[1] == 0.0 and np.isnan(got[2])
    assert abs(got[3] - 0.01 / 5) < 1e-15


def test_eoc_slope_power_laws():
    """Algorithm (ComputeSlopes): the slope of an exact power law C N^alpha is
    alpha; two points give log(D1/D0) / log(N1/N0); scaling N or D leaves it
    unchanged; for three points equally spaced in log N the least-squares
    slope is the end-to-end slope whatever the middle value."""
    ns = [32, 64, 128, 256]
    assert abs(oracle.eoc_slope(ns, [0.7 * n ** -0.45 for n in ns]) + 0.45) < 1e-13
    assert abs(oracle.eoc_slope([128, 512], [0.02, 0.005]) - math.log(0.25) / math.log(4)) < 1e-14
    ds = [0.3, 0.11, 0.07, 0.02]
    base = oracle.eoc_slope(ns, ds)
    assert abs(oracle.eoc_slope([3 * n for n in ns], [5 * d for d in ds]) - base) < 1e-13
    for mid in (0.01, 0.05, 0.2):
        assert abs(oracle.eoc_slope([64, 128, 256], [0.1, mid, 0.02]) - math.log(0.2) / math.log(4)) < 1e-14


def test_ensemble_mean_std_closed_forms():
    """eqs. (spectrum_mean), (spectrum_var): two samples give the midpoint and
    |a - b| / sqrt(2) (the 1/(M-1) normalisation); a constant column has
    zero spread; an affine map scales the spread by |alpha|; the Python
    standard library's sample statistics agree."""
    import statistics
    mean, std = oracle.ensemble_mean_std([[1.0, -2.0, 5.0], [3.0, 4.0, 5.0]])
    assert np.allclose(mean, [2.0, 1.0, 5.0], rtol=0, atol=1e-15)
    assert np.allclose(std, [2 / math.sqrt(2), 6 / math.sqrt(2), 0.0], rtol=1e-15, atol=0)
    rng = np.random.default_rng(22)
    x = rng.normal(size=(9, 4))
    mean, std = oracle.ensemble_mean_std(x)
    m2, s2 = oracle.ensemble_mean_std(-3.0 * x + 7.0)
    assert np.allclose(m2, -3.0 * mean + 7.0, rtol=1e-14) and np.allclose(s2, 3.0 * std, rtol=1e-13)
    for c in range(4):
        assert abs(mean[c] - statistics.fmean(x[:, c])) < 1e-15
        assert abs(std[c] - statistics.stdev(x[:, c])) < 1e-14


def test_compensation_of_k41_ranges_is_flat():
    """eqs. (compensatedE), (compensatedSF): a K41 spectrum C_Kol d^(2/3)
    kappa^(-5/3) (in units of u0^2) compensates to exactly 1, and a K41
    structure function C (d r)^(2/3) over physical lags r to the constant C,
    sample by sample with each sample's own d and u0."""
    n = 32
    c_kol = 1.5   # the K41 constant as the paper states it with eq. (compensatedE)
    d = np.array([0.3, 2.0e-3])
    u0 = np.array([0.05, 0.0125])
    kap = np.arange(n // 2 + 1, dtype=np.float64)
    ek = np.zeros((2, n // 2 + 1))
    ek[:, 1:] = (c_kol * np.cbrt(d ** 2)[:, None] * kap[1:] ** (-5.0 / 3.0)) * u0[:, None] ** 2
    ec = oracle.compensated_spectrum(ek, d, u0)
    assert np.max(np.abs(ec[:, 1:] - 1.0)) < 1e-14 and np.all(ec[:, 0] == 0.0)
    r = np.arange(1, n // 2 + 1) * 2 * math.pi / n
    s2 = 7.7 * np.cbrt((d[:, None] * r[None, :]) ** 2) * u0[:, None] ** 2
    sc = oracle.compensated_structure_function(s2, d, u0, n)
    assert np.max(np.abs(sc - 7.7)) < 1e-13


def test_taylor_green_field():
    """eq. (tgv_init_velo): divergence-free, and its values at sample nodes."""
    n = 8
    u = oracle.taylor_green(n)
    k = np.fft.fftfreq(n) * n
    KZ, KY, KX = np.meshgrid(k, k, k, indexing="ij")
    div = KX * np.fft.fftn(u[0]) + KY * np.fft.fftn(u[1]) + KZ * np.fft.fftn(u[2])
    assert np.max(np.abs(div)) < 1e-12
    # node (x, y, z) = (2, 1, 0) * 2 pi / 8
    x, y, z = 2 * math.pi * 2 / 8, 2 * math.pi * 1 / 8, 0.0
    assert abs(u[0, 0, 1, 2] - math.sin(x) * math.cos(y) * math.cos(z)) < 1e-15
    assert abs(u[1, 0, 1, 2] + math.cos(x) * math.sin(y) * math.cos(z)) < 1e-15
    assert u[2].max() == 0.0 and u[2].min() == 0.0


# ---------------------------------------------------------------- dissipation rate and Kolmogorov length
def test_energy_decay_rate_closed_forms():
    """The finite differences of the decay rate on series with closed-form
    differences: for E = C exp(-a t) on a uniform time grid of spacing h,
    the centred difference inside the series is a E(t_k) sinh(ah)/(ah), the
    forward difference at the start E(t_0)(1 - exp(-ah))/h and the backward
    one at the end E(t_K)(exp(ah) - 1)/h; centred differences of a
    quadratic are exact. Two columns (samples) are handled independently."""
    a, h, c = 3.0, 0.1, 2.5
    t = 0.7 + h * np.arange(6)
    e = c * np.exp(-a * t)
    d = oracle.energy_decay_rate(np.stack([e, 2 * e], axis=1), t)
    inner = a * e[1:-1] * math.sinh(a * h) / (a * h)
    assert np.max(np.abs(d[1:-1, 0] / inner - 1)) < 1e-13
    assert abs(d[0, 0] / (e[0] * (1 - math.exp(-a * h)) / h) - 1) < 1e-13
    assert abs(d[-1, 0] / (e[-1] * (math.exp(a * h) - 1) / h) - 1) < 1e-13
    assert np.max(np.abs(d[:, 1] - 2 * d[:, 0])) < 1e-15 * np.max(np.abs(d))
    q = 4.0 - 3.0 * t + 0.5 * t ** 2        # -dq/dt = 3 - t
    dq = oracle.energy_decay_rate(q, t)
    assert np.max(np.abs(dq[1:-1] - (3.0 - t[1:-1]))) < 1e-13


def test_dissipation_definition_closed_forms():
    """The definition before eq. (kolmogorov_microscale): for u / u0 = A TGV
    every component is a sum of |k|^2 = 3 modes with mean square A^2 / 8 (x
    and y components), so d = eps (3/4) A^2; a perturbation of eq.
    (alpha_perturbation) adds |k|^2 = 12 products of mean square (Y/8)^2 / 8,
    orthogonal to the TGV modes on the grid: d = eps (3/4 + amp^2 12 sum Y^2
    / 512) without projection. The spectral derivative equals the analytic
    derivative of the band-limited field."""
    n, u0, eps, amp = 16, 0.05, 1.0 / 400.0, 0.3
    d = oracle.dissipation_rate_definition(u0 * 0.8 * oracle.taylor_green(n), eps, u0)
    assert abs(d / (eps * 0.75 * 0.64) - 1) < 1e-13
    y = mc_inputs.draw_y(41, 1)[0]
    u = oracle.initial_velocity(n, u0, amp, y, False)
    d = oracle.dissipation_rate_definition(u, eps, u0)
    assert abs(d / (eps * (0.75 + amp ** 2 * 12 * np.sum(y ** 2) / 512)) - 1) < 1e-13
    # analytic gradient of the TGV on the grid: mean of |grad u|^2 / u0^2
    X, Y, Z = oracle.grid(n)
    gx = [np.cos(X) * np.cos(Y) * np.cos(Z), -np.sin(X) * np.sin(Y) * np.cos(Z), -np.sin(X) * np.cos(Y) * np.sin(Z)]
    gy = [np.sin(X) * np.sin(Y) * np.cos(Z), -np.cos(X) * np.cos(Y) * np.cos(Z), np.cos(X) * np.sin(Y) * np.sin(Z)]
    brute = eps * np.mean(sum(g * g for g in gx + gy))
    assert abs(oracle.dissipation_rate_definition(u0 * oracle.taylor_green(n), eps, u0) / brute - 1) < 1e-13


def test_dissipation_from_spectra_of_a_decaying_taylor_green_mode():
    """The paper's approximation, -d/dt sum_kappa E(kappa, t), for a TGV of
    amplitude exp(-3 eps t): its energy sits in shell 2 (62 modes, |k|^2 = 3
    for the 8 of the TGV), so sum_kappa E = (4 pi 3 / 62) KE with KE =
    exp(-6 eps t) / 8, a factor 0.608 below the kinetic energy per unit
    volume; the centred differences give 6 eps (4 pi 3/62)(1/8) exp(-6 eps
    t_k) sinh(6 eps h)/(6 eps h). The kinetic-energy form has no shell factor."""
    n, eps, h = 16, 1.0 / 50.0, 0.25
    u0 = np.array([0.05, 0.025])
    t = h * np.arange(5)
    amp = np.exp(-3 * eps * t)
    ek = np.stack([np.stack([oracle.energy_spectrum(u0[s] * a * oracle.taylor_green(n)) for s in range(2)])
                   for a in amp])
    ke = np.stack([[oracle.kinetic_energy(u0[s] * a * oracle.taylor_green(n)) for s in range(2)] for a in amp])
    d_spec = oracle.dissipation_from_spectra(ek, t, u0)
    d_ke = oracle.dissipation_from_kinetic_energy(ke, t, u0)
    r = 6 * eps
    inner = r * np.exp(-r * t[1:-1]) / 8 * math.sinh(r * h) / (r * h)
    factor = 4 * math.pi * 3 / 62
    for s in range(2):
        assert np.max(np.abs(d_ke[1:-1, s] / inner - 1)) < 1e-12
        assert np.max(np.abs(d_spec[1:-1, s] / (factor * inner) - 1)) < 1e-12
        assert abs(d_spec[0, s] / (factor * (1 - math.exp(-r * h)) / (8 * h)) - 1) < 1e-12


def test_kolmogorov_length_closed_form():
    """eq. (kolmogorov_microscale) with the ensemble-mean dissipation rate:
    eps = 1/2 and E[d] = 1/128 give eta = (16)^(1/4) = 2; eps = 0.01 with
    samples d = 0.01 (1 +- 0.3) gives 0.1; per record along the first axis."""
    assert abs(oracle.kolmogorov_length(0.5, [1.0 / 128.0]) - 2.0) < 1e-15
    eta = oracle.kolmogorov_length(0.01, [[0.013, 0.007], [1.0 / 128.0, 1.0 / 128.0]])
    assert abs(eta[0] - 0.1) < 1e-15
    assert abs(eta[1] - (1e-6 * 128.0) ** 0.25) < 1e-15
