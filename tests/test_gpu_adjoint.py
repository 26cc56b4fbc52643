"""Gradient of the ensemble-mean kinetic energy with respect to the 24 random
parameters per sample: the library's discrete adjoint against the oracle's
complex-step derivative, central finite differences of the GPU FP64 forward,
and structural properties.

Tolerances: FP64 adjoint vs complex step 1e-8 of max|dJ/dY| (both are exact
to rounding; the closed-form stabiliser is a ratio of small inner products,
which amplifies rounding). FP32 adjoint: stated per test, from the float
rounding of the forward states and of the reverse sweep.
"""
import json
import os

import numpy as np
import pytest
import torch

import mc_inputs
import oracle

pytestmark = pytest.mark.gpu
mc = pytest.importorskip("paper_2608_23786_amd")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def gpu_gradient(samples, precision, y, steps, every, stabiliser="closed_form"):
    ens = mc.Ensemble(samples, precision)
    ens.init(0, torch.from_numpy(y))
    ens.set_stabiliser(stabiliser)
    ck = ens.forward_ckpt(steps, every)
    dj, ke = ens.backward(steps, every, ck)
    return dj.cpu().numpy(), ke.cpu().numpy(), ens


def oracle_gradient(samples, y, steps, mode=oracle.MODE_KBC, params=None):
    m = len(samples)
    g = np.zeros((m, 24))
    ke = np.zeros(m)
    for s, smp in enumerate(samples):
        g[s] = oracle.ke_gradient_complex_step(smp.n, smp.u0, smp.re, smp.amp, y[s], smp.project, steps,
                                               params=params, mode=mode) / m
        ke[s] = oracle.ke_after(smp.n, smp.u0, smp.re, smp.amp, y[s], smp.project, steps, mode=mode)
    return g, ke


@pytest.mark.parametrize("steps,every", [(20, 6), (20, 20), (7, 1)])
def test_fp64_adjoint_matches_complex_step(steps, every):
    samples = [mc.Sample(8, 0.05, 100.0, 0.5, True), mc.Sample(8, 0.04, 60.0, 0.5, False)]
    y = mc_inputs.draw_y(21, 2)
    dj, ke, _ = gpu_gradient(samples, "f64", y, steps, every)
    g, ke_o = oracle_gradient(samples, y, steps)
    err = np.max(np.abs(dj - g)) / np.max(np.abs(g))
    print(f"steps {steps} every {every}: max |adjoint - complex step| / max = {err:.3e}")
    assert err < 1e-8
    assert np.max(np.abs(ke - ke_o) / ke_o) < 1e-12


def test_fp64_adjoint_16cubed():
    samples = [mc.Sample(16, 0.05, 200.0, 0.2, True)] * 2
    y = mc_inputs.draw_y(22, 2)
    dj, _, _ = gpu_gradient(samples, "f64", y, 40, 16)
    g, _ = oracle_gradient(samples, y, 40)
    assert np.max(np.abs(dj - g)) / np.max(np.abs(g)) < 1e-8


def test_fp32_adjoint_close_to_fp64_reference():
    samples = [mc.Sample(16, 0.05, 200.0, 0.2, True)] * 2
    y = mc_inputs.draw_y(22, 2)
    dj32, _, _ = gpu_gradient(samples, "f32s", y, 40, 10)
    g, _ = oracle_gradient(samples, y, 40)
    err = np.max(np.abs(dj32 - g)) / np.max(np.abs(g))
    print(f"fp32 adjoint: max rel err vs complex step = {err:.3e}")
    assert err < 1e-4


def test_central_differences_of_gpu_forward():
    """Central differences (h = 1e-3 on Y) of the GPU FP64 forward."""
    samples = [mc.Sample(16, 0.05, 200.0, 0.3, True), mc.Sample(16, 0.05, 200.0, 0.3, False)]
    steps, h = 30, 1e-3
    y = mc_inputs.draw_y(23, 2)
    dj, _, _ = gpu_gradient(samples, "f64", y, steps, 10)

    def J(yy):
        ens = mc.Ensemble(samples, "f64")
        ens.init(0, torch.from_numpy(yy))
        ens.step(steps)
        return float(ens.reduce()[:, 4].mean())

    for s, p in ((0, 0), (0, 11), (1, 5), (1, 23)):
        yp, ym = y.copy(), y.copy()
        yp[s, p] += h
        ym[s, p] -= h
        fd = (J(yp) - J(ym)) / (2 * h)
        assert abs(fd - dj[s, p]) <= 1e-6 * np.max(np.abs(dj)), (s, p, fd, dj[s, p])


def test_central_differences_at_128_cubed():
    """Rows of two waves: the adjoint pulls lambda and the recompute pushes
    populations by lane exchange. Central differences of the GPU FP64
    forward over both AA parities and two checkpoint segments."""
    samples = [mc.Sample(128, 0.0125, 1600.0, 0.3, True)]
    steps, every, h = 6, 3, 1e-3
    y = mc_inputs.draw_y(29, 1)
    dj, _, _ = gpu_gradient(samples, "f64", y, steps, every)

    def J(yy):
        ens = mc.Ensemble(samples, "f64")
        ens.init(0, torch.from_numpy(yy))
        ens.step(steps)
        return float(ens.reduce()[:, 4].mean())

    for p in (0, 11, 17):
        yp, ym = y.copy(), y.copy()
        yp[0, p] += h
        ym[0, p] -= h
        fd = (J(yp) - J(ym)) / (2 * h)
        print(f"p={p}: fd {fd:.6e} adjoint {dj[0, p]:.6e}")
        assert abs(fd - dj[0, p]) <= 1e-6 * np.max(np.abs(dj)), (p, fd, dj[0, p])


# ---------------------------------------------------------------- exact stabiliser
# The reverse step recomputes the forward t (the minimiser of the discrete
# H-function, eq. (kbc_entropy)) and differentiates it through dH/dt = 0.
# The oracle's complex step goes through its bisection root and Newton steps
# in complex arithmetic, a different route to the same derivative.

@pytest.mark.parametrize("steps,every", [(12, 5), (7, 1)])
def test_exact_stabiliser_fp64_adjoint_matches_complex_step(steps, every):
    """FP64; tolerance 1e-7 of max|dJ/dY|: the GPU's Newton stops at a
    step below 1e-8 of t (quadratic convergence leaves the root at rounding
    level), the rest as for the closed form."""
    samples = [mc.Sample(8, 0.05, 100.0, 0.5, True), mc.Sample(8, 0.04, 60.0, 0.5, False)]
    y = mc_inputs.draw_y(41, 2)
    dj, ke, _ = gpu_gradient(samples, "f64", y, steps, every, "exact")
    g, ke_o = oracle_gradient(samples, y, steps, oracle.MODE_EXACT)
    gk, _ = oracle_gradient(samples, y, steps)
    err = np.max(np.abs(dj - g)) / np.max(np.abs(g))
    gap = np.max(np.abs(gk - g)) / np.max(np.abs(g))
    print(f"exact stabiliser, steps {steps} every {every}: adjoint vs complex step {err:.3e} "
          f"(closed-form gradient differs by {gap:.3e})")
    assert err < 1e-7 and gap > 100 * err
    assert np.max(np.abs(ke - ke_o) / ke_o) < 1e-12


def test_exact_stabiliser_adjoint_is_fp64_only():
    """Near equilibrium the exact minimiser's change of f* does not vanish
    with dh (an oracle pin shows it), so its derivative grows like 1/|dh|;
    FP32 rounding of dh makes that derivative noise, and the library refuses
    the FP32 adjoint with the exact stabiliser."""
    samples = [mc.Sample(16, 0.05, 200.0, 0.2, True)]
    ens = mc.Ensemble(samples, "f32s")
    ens.init(0, torch.from_numpy(mc_inputs.draw_y(42, 1)))
    ens.set_stabiliser("exact")
    with pytest.raises(mc.MclbmError, match="ERR_UNSUPPORTED"):
        ens.forward_ckpt(4, 2)
    ens.set_stabiliser("closed_form")
    ck = ens.forward_ckpt(4, 2)
    dj, _ = ens.backward(4, 2, ck)
    assert torch.isfinite(dj).all()


def test_exact_stabiliser_central_differences_of_gpu_forward():
    """Central differences (h = 1e-3 on Y) of the GPU FP64 forward with the
    exact stabiliser, over both AA parities and three checkpoint segments."""
    samples = [mc.Sample(16, 0.05, 200.0, 0.3, True), mc.Sample(16, 0.05, 200.0, 0.3, False)]
    steps, h = 30, 1e-3
    y = mc_inputs.draw_y(43, 2)
    dj, _, _ = gpu_gradient(samples, "f64", y, steps, 10, "exact")

    def J(yy):
        ens = mc.Ensemble(samples, "f64")
        ens.init(0, torch.from_numpy(yy))
        ens.set_stabiliser("exact")
        ens.step(steps)
        return float(ens.reduce()[:, 4].mean())

    for s, p in ((0, 2), (0, 13), (1, 7), (1, 20)):
        yp, ym = y.copy(), y.copy()
        yp[s, p] += h
        ym[s, p] -= h
        fd = (J(yp) - J(ym)) / (2 * h)
        assert abs(fd - dj[s, p]) <= 1e-6 * np.max(np.abs(dj)), (s, p, fd, dj[s, p])


def test_projected_gradient_lies_in_the_range_of_the_projection():
    """With the Leray projection on, J depends on Y only through P Y, so dJ/dY
    is annihilated by I - P (P symmetric idempotent on the coefficients)."""
    n = 8
    basis = np.stack([oracle.perturbation(n, np.eye(24)[p]).ravel() for p in range(24)], axis=1)
    proj = np.stack([oracle.leray_project(oracle.perturbation(n, np.eye(24)[p])).ravel() for p in range(24)], axis=1)
    P = np.linalg.lstsq(basis, proj, rcond=None)[0]
    assert np.max(np.abs(P @ P - P)) < 1e-12 and np.max(np.abs(P - P.T)) < 1e-12
    samples = [mc.Sample(n, 0.05, 100.0, 0.5, True)]
    y = mc_inputs.draw_y(24, 1)
    dj, _, _ = gpu_gradient(samples, "f64", y, 10, 5)
    assert np.max(np.abs((np.eye(24) - P) @ dj[0])) < 1e-10 * np.max(np.abs(dj))


def test_autograd_function():
    samples = [mc.Sample(8, 0.05, 100.0, 0.5, True)] * 3
    ens = mc.Ensemble(samples, "f64")
    y = torch.from_numpy(mc_inputs.draw_y(25, 3)).requires_grad_(True)
    J = mc.EnsembleKE.apply(y, ens, 12, 5)
    J.backward()
    g, ke = oracle_gradient(samples, y.detach().numpy(), 12)
    assert abs(float(J.detach()) - ke.mean()) / ke.mean() < 1e-12
    assert np.max(np.abs(y.grad.numpy() - g)) / np.max(np.abs(g)) < 1e-8


def test_backward_leaves_the_final_forward_state():
    samples = [mc.Sample(8, 0.05, 100.0, 0.5, True)]
    y = mc_inputs.draw_y(26, 1)
    _, ke, ens = gpu_gradient(samples, "f64", y, 9, 4)
    assert ens.ticks == 9
    assert abs(float(ens.reduce()[0, 4]) - ke[0]) < 1e-15


def test_adjoint_argument_errors():
    ens = mc.Ensemble([mc.Sample(8, 0.05, 100.0, 0.5, True, 2)], "f64")
    ens.init(0)
    with pytest.raises(mc.MclbmError, match="ERR_UNSUPPORTED"):
        ens.forward_ckpt(4, 2)
    ens2 = mc.Ensemble([mc.Sample(8, 0.05, 100.0, 0.5, True)], "f64")
    ens2.init(0)
    ens2.step(1)
    with pytest.raises(mc.MclbmError, match="ERR_STATE"):
        ens2.forward_ckpt(4, 2)


@pytest.mark.parametrize("precision,tol", [("f64", 1e-8), ("f32s", 2e-3)])
def test_gradient_reference_32cubed_1000_steps(precision, tol):
    """2 RTGV samples at 32^3 over 1000 steps (the small reference case of the
    adjoint workload): GPU adjoint against the stored complex-step gradient.
    FP32 bound: each reverse step forms its outputs from sums of about 30
    float terms, a relative rounding of at most 30 * 2^-24 ~ 2e-6; the
    adjoint recursion of this viscous flow does not amplify, so over 1000
    steps the rounding adds up to at most ~2e-3 of the gradient (measured
    1.7e-5, the forward states' own FP32 error included)."""
    path = os.path.join(GOLDEN, "gradient_rtgv32_T1000.json")
    if not os.path.exists(path):
        pytest.skip("reference gradient not generated")
    ref = json.load(open(path))
    y = np.array(ref["y"])
    samples = [mc.Sample(ref["n"], ref["u0"], ref["re"], ref["amp"], ref["project"])] * ref["m"]
    assert np.array_equal(y, mc_inputs.draw_y(ref["seed"], ref["m"]))
    dj, ke, _ = gpu_gradient(samples, precision, y, ref["steps"], 50)
    g = np.array(ref["dJdY"])
    err = np.max(np.abs(dj - g)) / np.max(np.abs(g))
    print(f"{precision}: max |adjoint - reference| / max|reference| = {err:.3e}")
    assert err < tol
    assert np.max(np.abs(ke - np.array(ref["ke"])) / np.array(ref["ke"])) < (1e-12 if precision == "f64" else 1e-5)


def _nonequilibrium_state(n, q, seed):
    """An RTGV equilibrium times (1 + 2e-3 noise), f[n^3][q] (oracle layout):
    both the shear and the higher-order parts of f^neq are non-zero."""
    y = mc_inputs.draw_y(seed, 1)[0]
    f = oracle.init_populations(n, 0.05 * 16 / n, 0.5, y, True, q)
    return f * (1.0 + mc_inputs.random_populations(seed, f.shape, 2e-3))


@pytest.mark.parametrize("n,q,stabiliser,precision,tol", [
    (8, 27, "closed_form", "f64", 1e-12), (128, 27, "closed_form", "f64", 1e-12),
    (8, 19, "closed_form", "f64", 1e-12), (128, 19, "closed_form", "f64", 1e-12),
    (8, 27, "exact", "f64", 1e-11), (16, 19, "exact", "f64", 1e-11),
    (8, 27, "closed_form", "f32s", 1e-5), (128, 27, "closed_form", "f32s", 1e-5)])
def test_per_step_adjoint_is_the_transpose_of_the_step(n, q, stabiliser, precision, tol):
    """Dot-product test of one reverse step: <J v, lam> = <v, J^T lam> for
    random v and lam, with J the Jacobian of one collide-and-stream step at
    a non-equilibrium state. J v comes from the oracle's complex step
    (Im step(f + i h v) / h, h = 1e-30, exact to rounding) on its own copy
    of the state; J^T lam from the library's reverse-step kernel. n = 128
    rows span two waves (the row exchange of the forward kernel). The
    difference of the two dot products is measured against the sum of the
    absolute values of their terms, the scale of the rounding of either sum
    (random v and lam make the sums cancel by up to an order of magnitude).
    FP64: both sides exact to rounding (the closed-form stabiliser's ratio
    of inner products amplifies per-node rounding to ~1e-13), bound 1e-12
    (1e-11 for the exact stabiliser, whose Newton iterate is converged to
    rounding only up to its stopping rule). FP32: the reverse step in
    float on a float copy of the state, ~30-term sums per output, bound
    1e-5."""
    f = _nonequilibrium_state(n, q, 60 + n + q)
    ncell = n ** 3
    v = mc_inputs.random_populations(1000 + n, (ncell, q), 1.0)
    lam = mc_inputs.random_populations(2000 + n, (ncell, q), 1.0)
    u0, re = 0.05 * 16 / n, 50.0
    omega = oracle.omega_shear(oracle.lattice_viscosity(n, u0, re))
    mode = oracle.MODE_EXACT if stabiliser == "exact" else oracle.MODE_KBC
    h = 1e-30
    fz = f.astype(np.complex128) + 1j * h * v
    oracle.run(fz, n, 1, omega, mode=mode)
    jv = fz.imag / h
    lhs = float(np.sum(jv * lam))
    scale = float(np.sum(np.abs(jv * lam)))      # the size of the terms the two sums add

    ens = mc.Ensemble([mc.Sample(n, u0, re, 0.5, True)], precision, lattice=q)
    ens.init(0)
    ens.set_stabiliser(stabiliser)
    ens.set_state(0, torch.from_numpy(np.ascontiguousarray(f.T)).cuda())
    out = ens.step_vjp(torch.from_numpy(np.ascontiguousarray(lam.T)).reshape(-1).cuda())
    rhs = float(np.sum(v.T.reshape(-1) * out.cpu().numpy()))
    rel = abs(lhs - rhs) / scale
    print(f"n {n} D3Q{q} {stabiliser} {precision}: <Jv, lam> = {lhs:.15e}, <v, J^T lam> = {rhs:.15e}, "
          f"|difference| / sum |terms| {rel:.2e}, / |<Jv, lam>| {abs(lhs - rhs) / abs(lhs):.2e}")
    assert rel < tol
    # the state is not advanced
    assert ens.ticks == 0


@pytest.mark.parametrize("q,stabiliser", [(27, "closed_form"), (19, "closed_form"), (27, "exact")])
def test_step_vjp_keeps_the_collision_invariants(q, stabiliser):
    """Mass and momentum summed over the lattice are the same function of the
    state before and after a step (the collision conserves them per node,
    streaming moves populations), so the transpose maps the constant
    adjoints lam_i(x) = 1 and lam_i(x) = c_i,a to themselves, at any state,
    up to rounding (bound 1e-12: the closed-form stabiliser's ratio of inner
    products amplifies per-node rounding to ~1e-13)."""
    n = 16
    f = _nonequilibrium_state(n, q, 80 + q)
    c, _ = oracle.velocity_set(q)
    ens = mc.Ensemble([mc.Sample(n, 0.05, 100.0, 0.5, True)], "f64", lattice=q)
    ens.init(0)
    ens.set_stabiliser(stabiliser)
    ens.set_state(0, torch.from_numpy(np.ascontiguousarray(f.T)).cuda())
    for a in range(4):
        col = np.ones(q) if a == 3 else c[:, a].astype(np.float64)
        lam = np.repeat(col[:, None], n ** 3, axis=1).reshape(-1)
        out = ens.step_vjp(torch.from_numpy(lam).cuda()).cpu().numpy()
        assert np.max(np.abs(out - lam)) < 1e-12, a


def test_backward_refuses_checkpoints_of_an_earlier_forward():
    """Two forward passes on one ensemble, then the backward of the first:
    its checkpoints are not those of the state the ensemble now holds, and
    the library refuses (MCLBM_ERR_STATE) instead of mixing the two runs.
    The backward of the latest forward matches a single forward on a fresh
    ensemble bit for bit; a step after a forward also makes the backward
    refuse."""
    samples = [mc.Sample(8, 0.05, 100.0, 0.5, True)] * 2
    ens = mc.Ensemble(samples, "f64")
    y1 = torch.from_numpy(mc_inputs.draw_y(71, 2)).requires_grad_(True)
    y2 = torch.from_numpy(mc_inputs.draw_y(72, 2)).requires_grad_(True)
    j1 = mc.EnsembleKE.apply(y1, ens, 10, 4)
    j2 = mc.EnsembleKE.apply(y2, ens, 10, 4)
    with pytest.raises(Exception, match="ERR_STATE"):
        j1.backward()
    j2.backward()
    ref, _, _ = gpu_gradient(samples, "f64", y2.detach().numpy(), 10, 4)
    assert np.array_equal(y2.grad.numpy(), ref)
    ens.init(0, y1.detach())
    ck = ens.forward_ckpt(10, 4)
    ens.set_viscosity([1 / 100.0, 1 / 100.0])
    with pytest.raises(mc.MclbmError, match="state changed"):
        ens.backward(10, 4, ck)


def test_fp32_gradient_of_the_adjoint_workload_against_fp64():
    """Config 4 in the benchmarked shape: 8 x 128^3, FP32 forward over 1000
    steps with a checkpoint every 50 and the FP32 reverse sweep, against the
    FP64 adjoint of two of its samples over the same 1000 steps (the FP64
    adjoint matches the oracle's complex step to ~1e-12). J is the mean over
    the ensemble, so dJ/dY_m carries 1/M: the comparison is of M dJ/dY_m.
    Bound 2e-3 of the largest component, as for the 32^3 reference over 1000
    steps (linear accumulation of ~2e-6 per reverse step)."""
    wl = mc_inputs.WORKLOADS["adjoint128x8_f32"]
    g = wl.groups[0]
    y = mc_inputs.draw_y(wl.seed, wl.m)
    ens = mc.Ensemble([mc.Sample(g.n, g.u0, g.re, g.amp, g.project)] * wl.m, "f32s")
    ens.init(0, torch.from_numpy(y))
    ck = ens.forward_ckpt(wl.ticks, wl.save_every)
    dj32, ke32 = ens.backward(wl.ticks, wl.save_every, ck)
    dj32, ke32 = dj32.cpu().numpy() * wl.m, ke32.cpu().numpy()
    del ens, ck
    torch.cuda.empty_cache()
    pick = [0, wl.m - 1]
    ens = mc.Ensemble([mc.Sample(g.n, g.u0, g.re, g.amp, g.project)] * len(pick), "f64")
    ens.init(0, torch.from_numpy(np.ascontiguousarray(y[pick])))
    ck = ens.forward_ckpt(wl.ticks, wl.save_every)
    dj64, ke64 = ens.backward(wl.ticks, wl.save_every, ck)
    dj64, ke64 = dj64.cpu().numpy() * len(pick), ke64.cpu().numpy()
    del ens, ck
    torch.cuda.empty_cache()
    for k, s in enumerate(pick):
        err = np.max(np.abs(dj32[s] - dj64[k])) / np.max(np.abs(dj64[k]))
        kerr = abs(ke32[s] / ke64[k] - 1)
        print(f"sample {s}: FP32 gradient vs FP64 over 1000 steps {err:.2e}; KE {kerr:.2e}")
        assert err < 2e-3 and kerr < 2e-5
