"""Parity of the D3Q19 lattice (the paper's own velocity set) against the
oracle run on the same lattice (GPU tests).

The D3Q19 path shares the kernels of D3Q27, instantiated for 19 velocities:
the same class-wise shear split, the D3Q19 weights, 19 storage planes. The
oracle builds the collision from its own 19 x 19 moment basis. Tolerances as
for D3Q27: FP64 1e-12 relative L2 of u over a run, 2e-13 of max|f - w| for
single steps from non-equilibrium states; FP32 shifted 1e-5 relative L2 of u
and 2e-6 for single steps.
"""
import numpy as np
import pytest
import torch

import mc_inputs
import oracle

pytestmark = pytest.mark.gpu
mc = pytest.importorskip("paper_2608_23786_amd")

Q = 19


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def oracle_velocity(n, u0, re, amp, y, project, steps):
    om = oracle.omega_shear(oracle.lattice_viscosity(n, u0, re))
    f = oracle.init_populations(n, u0, amp, y, project, Q)
    oracle.run(f, n, steps, om)
    rho, u = oracle.moments(f, n)
    return rho, u, f


def to_gpu_layout(f, n):
    return torch.from_numpy(np.ascontiguousarray(f.T.reshape(Q, n, n, n))).cuda()


def from_gpu_layout(fg, n):
    return np.ascontiguousarray(fg.cpu().numpy().reshape(Q, n ** 3).T)


def ensemble(samples, precision):
    return mc.Ensemble(samples, precision, lattice=Q)


def test_lattice_argument_is_validated():
    with pytest.raises(mc.MclbmError, match="lattice"):
        mc.Ensemble([mc.Sample(8, 0.05, 100.0)], "f64", lattice=15)


def test_initial_state_matches_oracle():
    for precision, tol in (("f64", 1e-15), ("f32s", 1e-7)):
        n = 16
        y = mc_inputs.draw_y(5, 2)
        ens = ensemble([mc.Sample(n, 0.05, 100.0, 0.5, True), mc.Sample(n, 0.03, 100.0, 0.5, False)], precision)
        ens.init(0, torch.from_numpy(y))
        for s, (u0, proj) in enumerate(((0.05, True), (0.03, False))):
            fg = from_gpu_layout(ens.get_state(s), n)
            fo = oracle.init_populations(n, u0, 0.5, y[s], proj, Q)
            assert np.max(np.abs(fg - fo)) < tol


@pytest.mark.parametrize("precision,tol", [("f64", 2e-13), ("f32s", 2e-6)])
@pytest.mark.parametrize("nsteps", [1, 2, 3])
def test_single_steps_from_non_equilibrium_states(precision, tol, nsteps):
    n = 16
    rng = np.random.default_rng(200 + nsteps)
    _, w = oracle.velocity_set(Q)
    u = rng.uniform(-0.04, 0.04, (3, n, n, n))
    f = oracle.equilibrium_field(u, Q)
    f *= 1 + rng.uniform(-2e-3, 2e-3, f.shape)
    f = np.ascontiguousarray(f)
    ens = ensemble([mc.Sample(n, 0.05, 100.0)], precision)
    ens.init(0, torch.zeros(1, 24, dtype=torch.float64))
    ens.set_state(0, to_gpu_layout(f, n))
    ens.step(nsteps)
    fg = from_gpu_layout(ens.get_state(0), n)
    om = oracle.omega_shear(oracle.lattice_viscosity(n, 0.05, 100.0))
    oracle.run(f, n, nsteps, om)
    err = np.max(np.abs(fg - f)) / np.max(np.abs(f - w))
    print(f"D3Q19 {precision} {nsteps} steps: max |f_gpu - f_oracle| / max|f - w| = {err:.3e}")
    assert err < tol


def test_tgv32_fp64_matches_oracle_and_conserves():
    n, u0, re, steps = 32, 0.05, 100.0, 100
    ens = ensemble([mc.Sample(n, u0, re, 0.0, False)], "f64")
    ens.init(0, torch.zeros(1, 24, dtype=torch.float64))
    rec = ens.step(steps, record_every=10).cpu().numpy()
    _, u_g = (t.cpu().numpy() for t in ens.moments(0))
    _, u_o, _ = oracle_velocity(n, u0, re, 0.0, np.zeros(24), False, steps)
    err = rel_l2(u_g, u_o)
    print(f"D3Q19 TGV 32^3 FP64, 100 steps: rel L2(u) = {err:.3e}")
    assert err < 1e-12
    assert np.max(np.abs(rec[:, 0, 0] - n ** 3)) < 1e-9
    assert np.max(np.abs(rec[:, 0, 1:4])) < 1e-12


def test_rtgv_fp32_ensemble_matches_oracle():
    n, u0, re, amp, steps = 32, 0.05, 400.0, 0.05, 200
    y = mc_inputs.draw_y(2608, 3)
    ens = ensemble([mc.Sample(n, u0, re, amp, True)] * 3, "f32s")
    ens.init(0, torch.from_numpy(y))
    ens.step(steps)
    for s in range(3):
        _, u_g = (t.cpu().numpy() for t in ens.moments(s))
        _, u_o, _ = oracle_velocity(n, u0, re, amp, y[s], True, steps)
        err = rel_l2(u_g, u_o)
        print(f"D3Q19 sample {s}: rel L2(u) = {err:.3e}")
        assert err < 1e-5


def test_mixed_resolution_batch_and_records_match_oracle():
    specs = [(8, 4), (16, 2), (32, 1)]
    ticks = 32
    y = mc_inputs.draw_y(2609, len(specs))
    samples = [mc.Sample(n, 0.05 * 32 / n, 25.0 * n, 0.05, True, st) for n, st in specs]
    ens = ensemble(samples, "f64")
    ens.init(0, torch.from_numpy(y))
    rec = ens.step(ticks, record_every=8).cpu().numpy()
    for s, (n, st) in enumerate(specs):
        assert ens.steps(s) == ticks // st
        _, u_g = (t.cpu().numpy() for t in ens.moments(s))
        _, u_o, _ = oracle_velocity(n, 0.05 * 32 / n, 25.0 * n, 0.05, y[s], True, ticks // st)
        assert rel_l2(u_g, u_o) < 1e-12
        # the record of tick 8 describes the state after 8 // st steps
        _, _, f_o = oracle_velocity(n, 0.05 * 32 / n, 25.0 * n, 0.05, y[s], True, 8 // st)
        red_o = oracle.reductions(f_o, n)
        assert abs(rec[1, s, 0] - red_o[0]) < 1e-10
        assert abs(rec[1, s, 4] - red_o[4]) / red_o[4] < 1e-12


def run_state(precision, block, buf, nt, graphs):
    y = mc_inputs.draw_y(9, 3)
    ens = ensemble([mc.Sample(128, 0.0125, 1600.0, 0.3, True, 4), mc.Sample(256, 0.00625, 3200.0, 0.3, True, 1),
                    mc.Sample(16, 0.05, 100.0, 0.2, True, 4)], precision)
    ens.init(0, torch.from_numpy(y))
    ens.set_launch(block, 0, buf, nt)
    ens.use_graphs(graphs)
    ens.step(9)
    return [ens.get_state(s).cpu().numpy() for s in range(3)]


@pytest.mark.parametrize("precision", ["f32s", "f64"])
def test_results_do_not_depend_on_launch_shape(precision):
    """Bitwise equal states across block sizes (direct and lane-exchange
    x-shifts), addressing forms and graph capture."""
    ref = run_state(precision, 128, 0, 0, False)
    shapes = [(256, 1, 1, True), (512, 1, 0, False)]
    if precision == "f32s":
        shapes.append((1024, 1, 1, True))
    for block, buf, nt, graphs in shapes:
        out = run_state(precision, block, buf, nt, graphs)
        for s, (a, b) in enumerate(zip(ref, out)):
            assert np.array_equal(a, b), (block, buf, nt, graphs, s)


def test_sampled_steps_at_128_cubed():
    """Cells of a 128^3 FP32 sample after one step of either parity, against
    the oracle's collision of the neighbours' pre-step populations."""
    n = 128
    c, w = oracle.velocity_set(Q)
    ens = ensemble([mc.Sample(n, 0.0125, 1600.0, 0.05, True)], "f32s")
    ens.init(4)
    ens.set_launch(1024, 0, 1, 1)
    om = oracle.omega_shear(oracle.lattice_viscosity(n, 0.0125, 1600.0))
    rng = np.random.default_rng(19)
    for _ in range(2):
        cells = rng.choice(n ** 3, size=32, replace=False)
        x, yy, z = cells % n, (cells // n) % n, cells // (n * n)
        nb = np.zeros((32, Q), dtype=np.int64)
        for i in range(Q):
            nb[:, i] = (((z - c[i, 2]) % n) * n + (yy - c[i, 1]) % n) * n + (x - c[i, 0]) % n
        pre = ens.get_cells(0, nb.ravel()).cpu().numpy().reshape(32, Q, Q)
        ens.step(1)
        post = ens.get_cells(0, cells).cpu().numpy()
        expect = np.zeros_like(post)
        for k in range(32):
            for i in range(Q):
                expect[k, i] = oracle.collide(pre[k, i], om)[0][i]
        err = np.max(np.abs(post - expect)) / np.max(np.abs(expect - w))
        print(f"D3Q19 128^3 sampled step: {err:.3e}")
        assert err < 2e-6


def test_adjoint_matches_complex_step():
    samples = [mc.Sample(16, 0.05, 200.0, 0.3, True), mc.Sample(16, 0.05, 200.0, 0.3, False)]
    steps, every = 12, 5
    y = mc_inputs.draw_y(41, 2)
    ens = ensemble(samples, "f64")
    ens.init(0, torch.from_numpy(y))
    ck = ens.forward_ckpt(steps, every)
    dj, ke = (t.cpu().numpy() for t in ens.backward(steps, every, ck))
    g = np.zeros((2, 24))
    for s, smp in enumerate(samples):
        g[s] = oracle.ke_gradient_complex_step(16, 0.05, 200.0, 0.3, y[s], smp.project, steps, q=Q) / 2
        assert abs(ke[s] - oracle.ke_after(16, 0.05, 200.0, 0.3, y[s], smp.project, steps, q=Q)) < 1e-15
    err = np.max(np.abs(dj - g)) / np.max(np.abs(g))
    print(f"D3Q19 adjoint vs complex step: {err:.3e}")
    assert err < 1e-8


def test_exact_stabiliser_adjoint_matches_complex_step():
    """The adjoint of the exact stabiliser on D3Q19 (FP64) against the
    oracle's complex step through its bisection root; 1e-7 of max|dJ/dY| as
    on D3Q27."""
    samples = [mc.Sample(8, 0.05, 100.0, 0.5, True), mc.Sample(8, 0.04, 60.0, 0.5, False)]
    steps, every = 10, 4
    y = mc_inputs.draw_y(44, 2)
    ens = ensemble(samples, "f64")
    ens.init(0, torch.from_numpy(y))
    ens.set_stabiliser("exact")
    ck = ens.forward_ckpt(steps, every)
    dj = ens.backward(steps, every, ck)[0].cpu().numpy()
    g = np.zeros((2, 24))
    for s, smp in enumerate(samples):
        g[s] = oracle.ke_gradient_complex_step(8, smp.u0, smp.re, smp.amp, y[s], smp.project, steps, q=Q,
                                               mode=oracle.MODE_EXACT) / 2
    err = np.max(np.abs(dj - g)) / np.max(np.abs(g))
    print(f"D3Q19 exact-stabiliser adjoint vs complex step: {err:.3e}")
    assert err < 1e-7


def test_state_access_and_poison_use_19_planes():
    ens = ensemble([mc.Sample(8, 0.05, 100.0)] * 2, "f32s")
    ens.init(1)
    assert tuple(ens.get_state(0).shape) == (Q, 8, 8, 8)
    assert tuple(ens.get_cells(1, torch.arange(5)).shape) == (5, Q)
    with pytest.raises(mc.MclbmError, match="ERR_ARG"):
        ens.poison(0, 3, Q)
    ens.step(1)
    ens.poison(1, 17, 18)
    ens.step(1)
    assert ens.check() == 1
