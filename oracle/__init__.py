"""Oracle for the Monte Carlo KBC lattice Boltzmann hot path.

TEST INFRASTRUCTURE ONLY. Plain, slow, double-precision statements of what
the GPU library computes. Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package. It shares no code with the GPU
library; its inputs come from ``mc_inputs`` (random parameters only).

Contents and the passage each part follows:
  * parameter map (Table 1's omega from the viscosity; section "Randomized
    Taylor-Green vortex flow" for Re; Tables 2 and 3 for the paper's own
    Mach-number convention);
  * initial velocity, eqs. (tgv_init_velo), (alpha_perturbation),
    (initialRTGV), with the optional Leray projection done spectrally on
    the grid (a library FFT), and equilibrium populations,
    eq. (initialPopulations);
  * time stepping by the C++ part (``lbm_oracle.cpp``): eqs. (equilibrium),
    (bgkCollisionOp)-(momentDefin), (kbcCollision), (entropyControl),
    (kbc_entropy), (lbIteration);
  * moments rho = sum f, rho u = sum c f; kinetic energy per unit volume;
  * complex-step derivative of the ensemble-mean kinetic energy with
    respect to the 24 random parameters (Squire and Trapp 1998);
  * observables: energy spectrum, eqs. (dftCoeff), (energySpecDisc);
    structure function, Lemma (structureFunctionSpectral) / eq.
    (SF_single_spec2); 1-point Wasserstein distance between equal-size
    empirical laws by sorted rearrangement, eq. (wassersteinPermutations);
    the ensemble-mean relative L1 sample error, eq. (sample_error), and the
    least-squares convergence order of Algorithm (ComputeSlopes); empirical
    ensemble mean and standard deviation, eqs. (spectrum_mean) and
    (spectrum_var); sample-wise compensated spectrum and structure function,
    eqs. (compensatedE) and (compensatedSF);
  * the sample dissipation rate per unit volume as defined before eq.
    (kolmogorov_microscale) (viscosity times the mean squared velocity
    gradient, by spectral derivatives), its approximation the paper uses
    (minus the time derivative of the summed shell spectrum), the same
    derivative of the kinetic energy per unit volume, and the Kolmogorov
    length of eq. (kolmogorov_microscale).

Lattices: D3Q27 (q = 27, the default) and the paper's D3Q19 (q = 19).

Array conventions: fields are C-ordered [z][y][x] (x fastest); populations
f[cell][q] with, for D3Q27, i = 9*(cx+1) + 3*(cy+1) + (cz+1), and for D3Q19
the same order without the eight corner velocities; velocities u[3][z][y][x].
"""
import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t)


def lib():
    """Load liboracle.so, building it with g++ first if it is missing."""
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(path)
        _q = ctypes.c_int32
        L.oracle_velocity_set.argtypes = [_q, _ip, _dp]
        L.oracle_moment_basis.argtypes = [_q, _dp, _dp, _ip]
        L.oracle_equilibrium.argtypes = [_q, ctypes.c_double, _dp, _dp]
        L.oracle_collide.argtypes = [_q, _dp, ctypes.c_double, ctypes.c_int32, _dp, _dp, _dp, _dp]
        L.oracle_collide_z.argtypes = [_q, _dp, ctypes.c_double, ctypes.c_int32, _dp, _dp]
        L.oracle_run.argtypes = [_q, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, _dp, _dp,
                                 ctypes.c_int32]
        L.oracle_run_z.argtypes = [_q, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, _dp,
                                   ctypes.c_int32]
        L.oracle_init_field.argtypes = [_q, ctypes.c_int64, _dp, _dp]
        L.oracle_init_field_z.argtypes = [_q, ctypes.c_int64, _dp, _dp]
        for name in ("oracle_velocity_set", "oracle_moment_basis", "oracle_equilibrium", "oracle_collide",
                     "oracle_collide_z", "oracle_run", "oracle_run_z", "oracle_init_field", "oracle_init_field_z"):
            getattr(L, name).restype = ctypes.c_int32
        L.oracle_max_threads.restype = ctypes.c_int32
        _LIB = L
    return _LIB


# ---------------------------------------------------------------- lattice
LATTICES = (27, 19)


def _lat(q):
    if q not in LATTICES:
        raise ValueError(f"unknown lattice: {q} velocities")
    return q


def _ok(rc):
    assert rc == 1, "oracle call rejected its lattice"


def velocity_set(q=27):
    c = np.zeros((_lat(q), 3), dtype=np.int32)
    w = np.zeros(q)
    _ok(lib().oracle_velocity_set(q, _ptr(c, _ip), _ptr(w)))
    return c, w


def moment_basis(q=27):
    M = np.zeros((_lat(q), q))
    Minv = np.zeros((q, q))
    g = np.zeros(q, dtype=np.int32)
    _ok(lib().oracle_moment_basis(q, _ptr(M), _ptr(Minv), _ptr(g, _ip)))
    return M, Minv, g


def equilibrium(rho, u, q=27):
    u = np.ascontiguousarray(u, dtype=np.float64)
    feq = np.zeros(_lat(q))
    _ok(lib().oracle_equilibrium(q, float(rho), _ptr(u), _ptr(feq)))
    return feq


MODE_KBC, MODE_BGK, MODE_EXACT = 0, 1, 2


def collide(f, omega, mode=MODE_KBC):
    """One collision at one node (the lattice from len(f)). Returns (f*, gamma, ds, dh)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    q = _lat(f.shape[0])
    fs = np.zeros(q)
    ds = np.zeros(q)
    dh = np.zeros(q)
    g = np.zeros(1)
    _ok(lib().oracle_collide(q, _ptr(f), float(omega), int(mode), _ptr(fs), _ptr(g), _ptr(ds), _ptr(dh)))
    return fs, float(g[0]), ds, dh


def collide_complex(f, omega, mode=MODE_KBC):
    """collide() in complex arithmetic (complex steps): closed-form or exact
    stabiliser. Returns (f*, gamma)."""
    assert mode in (MODE_KBC, MODE_EXACT)
    f = np.ascontiguousarray(f, dtype=np.complex128)
    q = _lat(f.shape[0])
    fs = np.zeros(q, dtype=np.complex128)
    g = np.zeros(1, dtype=np.complex128)
    _ok(lib().oracle_collide_z(q, _ptr(f), float(omega), int(mode), _ptr(fs), _ptr(g)))
    return fs, g[0]


# ---------------------------------------------------------------- parameters
def lattice_viscosity(n, u0, re):
    """nu in lattice units for Re = U0 L / nu with L = n / (2 pi) lattice units."""
    return u0 * (n / (2.0 * math.pi)) / re


def omega_shear(nu):
    """Table 1: omega = 2 c_s^2 / (2 nu + c_s^2), c_s^2 = 1/3."""
    cs2 = 1.0 / 3.0
    return 2.0 * cs2 / (2.0 * nu + cs2)


def paper_table_row(n, ma, re, dx):
    """Relaxation time and physical time step of a row of Tables 2 and 3.

    Ma is relative to the lattice speed of sound, so the lattice velocity is
    Ma * c_s; the reference length 1 is 1/dx lattice units; the reference
    velocity is 1, so dt = dx * (lattice velocity)."""
    u_lu = ma * math.sqrt(1.0 / 3.0)
    nu = u_lu * (1.0 / dx) / re
    tau = 1.0 / omega_shear(nu)
    dt = dx * u_lu
    return tau, dt


# ---------------------------------------------------------------- initial data
def grid(n):
    x = 2.0 * math.pi * np.arange(n) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return X, Y, Z


def taylor_green(n):
    """eq. (tgv_init_velo) with unit amplitude, as [3][z][y][x]."""
    X, Y, Z = grid(n)
    return np.stack([np.sin(X) * np.cos(Y) * np.cos(Z), -np.cos(X) * np.sin(Y) * np.cos(Z), np.zeros_like(X)])


def perturbation(n, y):
    """eq. (alpha_perturbation) with coefficients y[24] (real or complex)."""
    X, Y, Z = grid(n)
    a = (np.sin, np.cos)
    y = np.asarray(y)
    s = np.zeros((3, n, n, n), dtype=np.result_type(y.dtype, np.float64))
    for al in range(3):
        for i in range(2):
            for j in range(2):
                for k in range(2):
                    s[al] += y[8 * al + 4 * i + 2 * j + k] * a[i](2 * X) * a[j](2 * Y) * a[k](2 * Z)
    return s / 8.0


def leray_project(v):
    """Remove the gradient part of a periodic field on the grid, spectrally.

    The projection is real-linear, so a complex field (complex-step input) is
    projected part by part: the FFT's own complex arithmetic must not mix the
    rounding of the real part into the imaginary part."""
    if np.iscomplexobj(v):
        return leray_project(np.ascontiguousarray(v.real)) + 1j * leray_project(np.ascontiguousarray(v.imag))
    n = v.shape[1]
    k = np.fft.fftfreq(n) * n
    KZ, KY, KX = np.meshgrid(k, k, k, indexing="ij")
    K = (KX, KY, KZ)
    k2 = KX ** 2 + KY ** 2 + KZ ** 2
    k2[0, 0, 0] = 1.0
    vh = [np.fft.fftn(v[a]) for a in range(3)]
    div = K[0] * vh[0] + K[1] * vh[1] + K[2] * vh[2]
    return np.stack([np.fft.ifftn(vh[a] - K[a] * div / k2).real for a in range(3)])


def initial_velocity(n, u0, amp, y, project):
    """u0 = U0 [TGV + amp * P s(Y)] (section "Discretization and well-prepared
    initial data"; the projection P is optional as in the numerics section)."""
    s = perturbation(n, y)
    if project:
        s = leray_project(s)
    return u0 * (taylor_green(n) + amp * s)


def equilibrium_field(u, q=27):
    """eq. (initialPopulations): f = f^eq(1, u) at every node -> f[ncell][q]."""
    n = u.shape[1]
    ncell = n ** 3
    if np.iscomplexobj(u):
        uu = np.ascontiguousarray(u.reshape(3, ncell), dtype=np.complex128)
        f = np.zeros((ncell, _lat(q)), dtype=np.complex128)
        _ok(lib().oracle_init_field_z(q, ncell, _ptr(uu), _ptr(f)))
    else:
        uu = np.ascontiguousarray(u.reshape(3, ncell), dtype=np.float64)
        f = np.zeros((ncell, _lat(q)))
        _ok(lib().oracle_init_field(q, ncell, _ptr(uu), _ptr(f)))
    return f


def init_populations(n, u0, amp, y, project, q=27):
    return equilibrium_field(initial_velocity(n, u0, amp, y, project), q)


# ---------------------------------------------------------------- time stepping
def run(f, n, steps, omega, mode=MODE_KBC, threads=0, gamma_stats=False):
    """Advance f[ncell][q] in place by `steps` steps (the lattice from the
    second dimension); optionally return the per-step (min, max, mean) of gamma."""
    q = _lat(f.shape[1])
    assert f.shape == (n ** 3, q) and f.flags.c_contiguous
    gs = np.zeros((max(steps, 1), 3)) if gamma_stats else None
    if np.iscomplexobj(f):
        assert mode in (MODE_KBC, MODE_EXACT) and not gamma_stats
        _ok(lib().oracle_run_z(q, n, steps, float(omega), int(mode), _ptr(f), int(threads)))
    else:
        _ok(lib().oracle_run(q, n, steps, float(omega), int(mode), _ptr(f), _ptr(gs) if gs is not None else None,
                             int(threads)))
    return gs[:steps] if gs is not None else None


def max_threads():
    return int(lib().oracle_max_threads())


# ---------------------------------------------------------------- moments and reductions
def moments(f, n):
    """rho[z][y][x], u[3][z][y][x] with rho = sum f, rho u = sum c f."""
    c, _ = velocity_set(f.shape[1])
    rho = f.sum(axis=1)
    j = f @ c.astype(np.float64)
    u = (j / rho[:, None]).T
    return rho.reshape(n, n, n), u.reshape(3, n, n, n)


def kinetic_energy(u):
    """Mean of |u|^2 / 2 over the nodes (energy per unit volume of u).
    Uses u.u without conjugation so that complex steps carry derivatives."""
    return 0.5 * np.mean(u[0] * u[0] + u[1] * u[1] + u[2] * u[2])


def reductions(f, n):
    """mass, jx, jy, jz (sums over nodes), kinetic energy."""
    c, _ = velocity_set(f.shape[1])
    rho, u = moments(f, n)
    j = f @ c.astype(np.float64)
    return np.array([rho.sum(), j[:, 0].sum(), j[:, 1].sum(), j[:, 2].sum(), kinetic_energy(u)])


# ---------------------------------------------------------------- gradient reference
def ke_gradient_complex_step(n, u0, re, amp, y, project, steps, h=1e-30, threads=0, params=None, q=27,
                             mode=MODE_KBC):
    """d KE(T) / d Y_p for one sample by the complex step Im KE(Y + i h e_p) / h
    (closed-form or exact stabiliser)."""
    omega = omega_shear(lattice_viscosity(n, u0, re))
    params = range(24) if params is None else params
    grad = np.zeros(24)
    for p in params:
        yc = np.asarray(y, dtype=np.complex128).copy()
        yc[p] += 1j * h
        f = init_populations(n, u0, amp, yc, project, q)
        run(f, n, steps, omega, mode=mode, threads=threads)
        _, u = moments(f, n)
        grad[p] = kinetic_energy(u).imag / h
    return grad


def ke_after(n, u0, re, amp, y, project, steps, threads=0, q=27, mode=MODE_KBC):
    omega = omega_shear(lattice_viscosity(n, u0, re))
    f = init_populations(n, u0, amp, np.asarray(y, dtype=np.float64), project, q)
    run(f, n, steps, omega, mode=mode, threads=threads)
    _, u = moments(f, n)
    return float(kinetic_energy(u))


# ---------------------------------------------------------------- observables
def energy_spectrum(u):
    """eq. (energySpecDisc): E(kappa) for kappa = 0..N/2 from eq. (dftCoeff)
    coefficients; modes whose rounded |k| exceeds N/2 are not counted."""
    n = u.shape[1]
    uh = np.stack([np.fft.fftn(u[a]) / n ** 3 for a in range(3)])
    phi = np.sum(np.abs(uh) ** 2, axis=0)
    k = np.fft.fftfreq(n) * n
    k[k == -n // 2] = n // 2   # index set {-N/2+1, ..., N/2}
    KZ, KY, KX = np.meshgrid(k, k, k, indexing="ij")
    kmag2 = KX ** 2 + KY ** 2 + KZ ** 2
    shell = np.floor(np.sqrt(kmag2) + 0.5).astype(np.int64)
    E = np.zeros(n // 2 + 1)
    for kap in range(n // 2 + 1):
        sel = shell == kap
        cnt = np.count_nonzero(sel)
        if cnt:
            E[kap] = 4.0 * math.pi / cnt * np.sum(0.5 * kmag2[sel] * phi[sel])
    return E


def autocorrelation(u):
    """eq. (SF_approx_spec5): R_h = N^-d F^-1(sum_i |F u_i|^2)_h."""
    n = u.shape[1]
    psd = sum(np.abs(np.fft.fftn(u[a])) ** 2 for a in range(3))
    return np.fft.ifftn(psd).real / n ** 3


def structure_function(u):
    """eq. (SF_single_spec2): S2(r) for r = 1..N/2 over the shells C_r of lags
    (minimum image) whose Euclidean length rounds to r."""
    n = u.shape[1]
    R = autocorrelation(u)
    h = np.fft.fftfreq(n) * n
    h[h == -n // 2] = n // 2
    HZ, HY, HX = np.meshgrid(h, h, h, indexing="ij")
    rr = np.floor(np.sqrt(HX ** 2 + HY ** 2 + HZ ** 2) + 0.5).astype(np.int64)
    S = np.zeros(n // 2)
    for r in range(1, n // 2 + 1):
        sel = rr == r
        S[r - 1] = np.mean(2.0 * (R[0, 0, 0] - R[sel]))
    return S


def wasserstein1_equal_weights(a, b):
    """W1 between two empirical laws with the same number of equal-weight
    atoms on the real line: mean |sorted(a) - sorted(b)|."""
    a = np.sort(np.asarray(a, dtype=np.float64))
    b = np.sort(np.asarray(b, dtype=np.float64))
    assert a.shape == b.shape
    return float(np.mean(np.abs(a - b)))


def sample_error_l1(a, b):
    """eq. (sample_error): the mean over the M samples of the relative L1
    distance between sample m at resolution N (a) and sample m of the
    reference resolution (b, drawn from the same Y_m), over the common nodes.
    a, b: point values [M][3][G]. Returns four values: one per velocity
    component (|.| the absolute value of that component) and one for the
    velocity vector (|.| its Euclidean length). A sample whose reference
    values of a quantity are all zero, where the definition has no value,
    makes it +inf (NaN if its own values are all zero too)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    assert a.shape == b.shape and a.ndim == 3 and a.shape[1] == 3
    m, _, g = a.shape
    out = np.zeros(4)
    with np.errstate(divide="ignore", invalid="ignore"):
        for s in range(m):
            for c in range(3):
                num = sum(abs(a[s, c, k] - b[s, c, k]) for k in range(g))
                den = sum(abs(b[s, c, k]) for k in range(g))
                out[c] += np.float64(num) / np.float64(den)
            num = sum(math.sqrt(sum((a[s, c, k] - b[s, c, k]) ** 2 for c in range(3))) for k in range(g))
            den = sum(math.sqrt(sum(b[s, c, k] ** 2 for c in range(3))) for k in range(g))
            out[3] += np.float64(num) / np.float64(den)
    return out / m


def eoc_slope(ns, ds):
    """Algorithm (ComputeSlopes): the experimental order of convergence at one
    time is the slope of the least-squares line through the points
    (log N, log D_N) of the distances D_N to the reference resolution."""
    return float(np.polyfit(np.log(np.asarray(ns, dtype=np.float64)),
                            np.log(np.asarray(ds, dtype=np.float64)), 1)[0])


def ensemble_mean_std(x):
    """eqs. (spectrum_mean), (spectrum_var): per column of x[M][K], the
    empirical mean (1/M) sum_m x_m and the empirical standard deviation
    sqrt(1/(M-1) sum_m (x_m - mean)^2) (M >= 2)."""
    x = np.asarray(x, dtype=np.float64)
    m, k = x.shape
    assert m >= 2
    mean = np.zeros(k)
    std = np.zeros(k)
    for c in range(k):
        mean[c] = sum(x[i, c] for i in range(m)) / m
        std[c] = math.sqrt(sum((x[i, c] - mean[c]) ** 2 for i in range(m)) / (m - 1))
    return mean, std


KOLMOGOROV_CONSTANT = 1.5   # C_Kol of eq. (compensatedE)


def compensated_spectrum(ek, d, u0):
    """eq. (compensatedE), sample by sample: E^c_m(kappa) = kappa^(5/3)
    E_m(kappa) / (C_Kol d_m^(2/3)), with E_m in units of u0^2 (the library's
    spectra are in lattice units) and d_m the sample's dissipation rate in
    the same physical units; d^(2/3) taken as the cube root of d^2.
    ek[M][N/2+1] for kappa = 0..N/2, d[M], u0[M]."""
    ek = np.asarray(ek, dtype=np.float64)
    out = np.zeros_like(ek)
    for m in range(ek.shape[0]):
        d23 = np.cbrt(d[m] * d[m])
        for kap in range(ek.shape[1]):
            out[m, kap] = kap ** (5.0 / 3.0) * (ek[m, kap] / u0[m] ** 2) / (KOLMOGOROV_CONSTANT * d23)
    return out


def compensated_structure_function(s2, d, u0, n):
    """eq. (compensatedSF), sample by sample: S^{2,c}_m(r) = S2_m(r) /
    (d_m r)^(2/3) with S2_m in units of u0^2 and r the physical lag
    r_lattice * 2 pi / n, r_lattice = 1..N/2. s2[M][N/2], d[M], u0[M]."""
    s2 = np.asarray(s2, dtype=np.float64)
    out = np.zeros_like(s2)
    for m in range(s2.shape[0]):
        for j in range(s2.shape[1]):
            r = (j + 1) * 2.0 * math.pi / n
            out[m, j] = (s2[m, j] / u0[m] ** 2) / np.cbrt((d[m] * r) ** 2)
    return out


# ---------------------------------------------------------------- dissipation rate and Kolmogorov length
def state_time(steps, n, u0):
    """Physical time after `steps` lattice steps: one step is dt = dx * u0 with
    dx = 2 pi / n (box of side 2 pi, unit reference velocity), the time step
    of Tables 2 and 3 for a lattice velocity u0."""
    return np.asarray(steps, dtype=np.float64) * (2.0 * math.pi / n) * u0


def energy_decay_rate(energy, t):
    """-dE/dt of a series E(t_k), k = 0..K-1 (K >= 2; the first axis is
    time): centred differences (E_{k+1} - E_{k-1}) / (t_{k+1} - t_{k-1})
    inside the series, one-sided differences at its two ends."""
    e = np.asarray(energy, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    k_len = e.shape[0]
    assert k_len >= 2 and t.shape == (k_len,)
    out = np.zeros_like(e)
    for k in range(k_len):
        lo = max(k - 1, 0)
        hi = min(k + 1, k_len - 1)
        out[k] = -(e[hi] - e[lo]) / (t[hi] - t[lo])
    return out


def dissipation_from_spectra(ek_series, t, u0):
    """The paper's approximation of the sample dissipation rate (the
    definition before eq. (kolmogorov_microscale)): d_m(t) = -d/dt of
    sum_kappa E_m(kappa, t), the shell spectrum of eq. (energySpecDisc)
    summed over kappa = 0..N/2, in units of u0^2 (velocities in units of
    the reference velocity). ek_series[K][M][N/2+1] in lattice units, t[K]
    physical times, u0[M]. Returns d[K][M]."""
    ek = np.asarray(ek_series, dtype=np.float64)
    k_len, m, _ = ek.shape
    total = np.zeros((k_len, m))
    for k in range(k_len):
        for s in range(m):
            total[k, s] = sum(ek[k, s, kap] for kap in range(ek.shape[2])) / u0[s] ** 2
    return energy_decay_rate(total, t)


def dissipation_from_kinetic_energy(ke_series, t, u0):
    """-d/dt of the kinetic energy per unit volume, mean |u|^2 / 2 over the
    nodes (the Parseval sum over every mode, corner modes included), in
    units of u0^2. ke_series[K][M] in lattice units, t[K], u0[M]."""
    ke = np.asarray(ke_series, dtype=np.float64)
    return energy_decay_rate(ke / np.asarray(u0, dtype=np.float64)[None, :] ** 2, t)


def dissipation_rate_definition(u, eps, u0):
    """The sample dissipation rate per unit volume as the paper defines it,
    d = eps / |Omega| * ||grad u||^2_{L^2(Omega)}, with eps = 1/Re the
    viscosity in units of the reference length and velocity and u in units
    of u0 on the box [0, 2 pi)^3; the derivatives of the trigonometric
    interpolant of the grid field (spectral: d/dx_a of exp(i k.x) is
    i k_a exp(i k.x), k in {-N/2+1, .., N/2}^3), so that |Omega|^-1
    ||grad u||^2 = sum_k |k|^2 Phi(k) with Phi of eq. (dftCoeff)."""
    n = u.shape[1]
    k = np.fft.fftfreq(n) * n
    k[k == -n // 2] = n // 2
    KZ, KY, KX = np.meshgrid(k, k, k, indexing="ij")
    k2 = KX ** 2 + KY ** 2 + KZ ** 2
    phi = sum(np.abs(np.fft.fftn(u[a] / u0) / n ** 3) ** 2 for a in range(3))
    return float(eps * np.sum(k2 * phi))


def kolmogorov_length(eps, d):
    """eq. (kolmogorov_microscale): eta(t) = (eps^3 / E[d(t)])^(1/4) with
    E[d] the empirical mean of the sample dissipation rates d[..., M] over
    the last axis."""
    d = np.asarray(d, dtype=np.float64)
    mean = np.sum(d, axis=-1) / d.shape[-1]
    return (eps ** 3 / mean) ** 0.25
