"""Parity of the HIP path against the oracle (GPU tests).

Inputs are seeded and synthetic; every comparison runs the oracle on the same
inputs. Tolerances:
  * FP64 path: relative L2 of u <= 1e-12 after 100 steps (summation order
    and FMA contraction differ between the two implementations; errors grow
    slowly with the number of steps).
  * FP32 shifted path: relative L2 of u <= 1e-5 (the target of the hot
    path) after the stated number of steps.
"""
import numpy as np
import pytest
import torch

import mc_inputs
import oracle

pytestmark = pytest.mark.gpu

mc = pytest.importorskip("paper_2608_23786_amd")


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def oracle_velocity(n, u0, re, amp, y, project, steps):
    om = oracle.omega_shear(oracle.lattice_viscosity(n, u0, re))
    f = oracle.init_populations(n, u0, amp, y, project)
    oracle.run(f, n, steps, om)
    rho, u = oracle.moments(f, n)
    return rho, u, f


def gpu_velocity(ens, s):
    rho, u = ens.moments(s)
    return rho.cpu().numpy(), u.cpu().numpy()


def to_gpu_layout(f, n):
    """oracle f[cell][27] -> [27][n][n][n] (device, float64)"""
    return torch.from_numpy(np.ascontiguousarray(f.T.reshape(27, n, n, n))).cuda()


def from_gpu_layout(fg, n):
    return np.ascontiguousarray(fg.cpu().numpy().reshape(27, n ** 3).T)


# ------------------------------------------------------------------ config 1
def test_tgv32_fp64_matches_oracle_and_conserves():
    """Single-sample plain method: 32^3, FP64, TGV U0 = 0.05, Re = 100, 100 steps."""
    n, u0, re, steps = 32, 0.05, 100.0, 100
    ens = mc.Ensemble([mc.Sample(n, u0, re)], "f64")
    ens.init(0, torch.zeros(1, 24, dtype=torch.float64))
    rec = ens.step(steps, record_every=1).cpu().numpy()[:, 0, :]
    red_end = ens.reduce().cpu().numpy()[0]
    rho_g, u_g = gpu_velocity(ens, 0)

    om = oracle.omega_shear(oracle.lattice_viscosity(n, u0, re))
    f = oracle.init_populations(n, u0, 0.0, np.zeros(24), False)
    ke_o = [oracle.kinetic_energy(oracle.moments(f, n)[1])]
    for k in range(steps):
        oracle.run(f, n, 1, om)
        ke_o.append(oracle.kinetic_energy(oracle.moments(f, n)[1]))
    rho_o, u_o = oracle.moments(f, n)
    err = rel_l2(u_g, u_o)
    print(f"tgv32 f64: rel L2(u) = {err:.3e}")
    assert err < 1e-12
    assert np.max(np.abs(rho_g - rho_o)) < 1e-13
    # kinetic energy at every step (records hold the state at the start of each tick)
    ke_g = np.append(rec[:, 4], red_end[4])
    assert np.max(np.abs(ke_g - np.array(ke_o)) / ke_o[0]) < 1e-12
    # viscous decay (the first steps carry the acoustic transient of the rho = 1 start)
    assert ke_g[-1] < ke_g[50] < ke_g[0]
    # exact conservation of mass and momentum
    mass = np.append(rec[:, 0], red_end[0])
    assert np.max(np.abs(mass - n ** 3)) < 1e-9
    mom = np.vstack([rec[:, 1:4], red_end[1:4]])
    assert np.max(np.abs(mom)) < 1e-12


# ------------------------------------------------------------------ single steps from random states
@pytest.mark.parametrize("precision,tol", [("f64", 2e-13), ("f32s", 2e-6)])
@pytest.mark.parametrize("nsteps", [1, 2, 3])
def test_single_steps_from_non_equilibrium_states(precision, tol, nsteps):
    """Strongly non-equilibrium states (0.2 % noise on every population).
    FP64 bound: the oracle works on unshifted f (~0.3) through dense 27 x 27
    moment products; perturbing its input by one rounding unit moves its own
    one-step output by up to 7e-14 of max|f - w| on these states, so the
    bound is 2e-13 of max|f - w|. FP32 bound: float rounding of g = f - w."""
    n = 16
    rng = np.random.default_rng(100 + nsteps)
    c, w = oracle.velocity_set()
    u = rng.uniform(-0.04, 0.04, (3, n, n, n))
    f = oracle.equilibrium_field(u)
    f *= 1 + rng.uniform(-2e-3, 2e-3, f.shape)
    f = np.ascontiguousarray(f)
    ens = mc.Ensemble([mc.Sample(n, 0.05, 100.0)], precision)
    ens.init(0, torch.zeros(1, 24, dtype=torch.float64))
    ens.set_state(0, to_gpu_layout(f, n))
    ens.step(nsteps)
    fg = from_gpu_layout(ens.get_state(0), n)
    om = oracle.omega_shear(oracle.lattice_viscosity(n, 0.05, 100.0))
    oracle.run(f, n, nsteps, om)
    err = np.max(np.abs(fg - f)) / np.max(np.abs(f - w))
    print(f"{precision} {nsteps} steps: max |f_gpu - f_oracle| / max|f - w| = {err:.3e}")
    assert err < tol


# ------------------------------------------------------------------ RTGV ensembles
def test_rtgv_fp32_ensemble_matches_oracle():
    """4 RTGV samples at 32^3 in one launch, FP32 shifted, 200 steps."""
    n, u0, re, amp, steps = 32, 0.05, 400.0, 0.05, 200
    y = mc_inputs.draw_y(2608, 4)
    ens = mc.Ensemble([mc.Sample(n, u0, re, amp, True)] * 4, "f32s")
    ens.init(0, torch.from_numpy(y))
    ens.step(steps)
    for s in range(4):
        _, u_g = gpu_velocity(ens, s)
        _, u_o, _ = oracle_velocity(n, u0, re, amp, y[s], True, steps)
        err = rel_l2(u_g, u_o)
        print(f"sample {s}: rel L2(u) = {err:.3e}")
        assert err < 1e-5


@pytest.mark.slow
def test_rtgv64_fp32_1000_steps_within_target():
    """The 64^3 RTGV sample of the 64-sample workload (U0 0.025, Re 1600,
    projected, seed 2608, sample 0) after 1000 steps: FP32 shifted
    populations against the FP64 oracle, relative L2 of u <= 1e-5."""
    n, u0, re, amp, steps = 64, 0.025, 1600.0, 0.05, 1000
    y = mc_inputs.draw_y(2608, 2)
    ens = mc.Ensemble([mc.Sample(n, u0, re, amp, True)] * 2, "f32s")
    ens.init(0, torch.from_numpy(y))
    ens.step(steps)
    _, u_g = gpu_velocity(ens, 0)
    _, u_o, _ = oracle_velocity(n, u0, re, amp, y[0], True, steps)
    err = rel_l2(u_g, u_o)
    print(f"64^3 RTGV, 1000 steps, FP32: rel L2(u) = {err:.3e}, max rel = {np.max(np.abs(u_g - u_o)) / np.max(np.abs(u_o)):.3e}")
    assert err < 1e-5


def test_fp64_rtgv_unprojected_matches_oracle():
    n, u0, re, amp, steps = 16, 0.05, 200.0, 0.4, 60
    y = mc_inputs.draw_y(11, 2)
    ens = mc.Ensemble([mc.Sample(n, u0, re, amp, False), mc.Sample(n, u0, re, amp, True)], "f64")
    ens.init(0, torch.from_numpy(y))
    ens.step(steps)
    for s, proj in ((0, False), (1, True)):
        _, u_g = gpu_velocity(ens, s)
        _, u_o, _ = oracle_velocity(n, u0, re, amp, y[s], proj, steps)
        assert rel_l2(u_g, u_o) < 1e-12


def test_initial_state_matches_oracle():
    for precision, tol in (("f64", 1e-15), ("f32s", 1e-7)):
        n = 16
        y = mc_inputs.draw_y(5, 2)
        ens = mc.Ensemble([mc.Sample(n, 0.05, 100.0, 0.5, True), mc.Sample(n, 0.03, 100.0, 0.5, False)], precision)
        ens.init(0, torch.from_numpy(y))
        for s, (u0, proj) in enumerate(((0.05, True), (0.03, False))):
            fg = from_gpu_layout(ens.get_state(s), n)
            fo = oracle.init_populations(n, u0, 0.5, y[s], proj)
            assert np.max(np.abs(fg - fo)) < tol


def test_seeded_parameters_follow_splitmix64():
    ens = mc.Ensemble([mc.Sample(8, 0.05, 100.0)] * 3, "f32s")
    ens.init(2608)
    assert np.array_equal(ens.y().numpy(), mc_inputs.draw_y(2608, 3))


def test_mixed_resolution_batch_matches_oracle():
    """Uneven batch 8^3 / 16^3 / 32^3 at strides 4:2:1 in one launch per tick."""
    specs = [(8, 4), (16, 2), (32, 1), (16, 2)]
    ticks = 48
    y = mc_inputs.draw_y(2609, len(specs))
    samples = [mc.Sample(n, 0.05 * 32 / n, 25.0 * n, 0.05, True, st) for n, st in specs]
    ens = mc.Ensemble(samples, "f64")
    ens.init(0, torch.from_numpy(y))
    ens.step(ticks)
    for s, (n, st) in enumerate(specs):
        assert ens.steps(s) == ticks // st
        _, u_g = gpu_velocity(ens, s)
        _, u_o, _ = oracle_velocity(n, 0.05 * 32 / n, 25.0 * n, 0.05, y[s], True, ticks // st)
        assert rel_l2(u_g, u_o) < 1e-12


def test_records_match_reduce_and_oracle():
    n, steps = 16, 12
    y = mc_inputs.draw_y(3, 2)
    ens = mc.Ensemble([mc.Sample(n, 0.05, 300.0, 0.2, True)] * 2, "f64")
    ens.init(0, torch.from_numpy(y))
    rec = ens.step(steps, record_every=4).cpu().numpy()
    assert rec.shape == (3, 2, 8)
    for k, t in enumerate((0, 4, 8)):
        for s in range(2):
            _, u_o, f_o = oracle_velocity(n, 0.05, 300.0, 0.2, y[s], True, t)
            red_o = oracle.reductions(f_o, n)
            assert abs(rec[k, s, 0] - red_o[0]) < 1e-10
            assert np.max(np.abs(rec[k, s, 1:4] - red_o[1:4])) < 1e-12
            assert abs(rec[k, s, 4] - red_o[4]) / red_o[4] < 1e-12
            assert rec[k, s, 5] <= rec[k, s, 7] <= rec[k, s, 6]
    # gamma statistics of the closed form on a state, against the oracle's per-node gamma
    om = oracle.omega_shear(oracle.lattice_viscosity(n, 0.05, 300.0))
    f = oracle.init_populations(n, 0.05, 0.2, y[0], True)
    oracle.run(f, n, 4, om)
    gs = oracle.run(f.copy(), n, 1, om, gamma_stats=True)[0]
    assert abs(rec[1, 0, 5] - gs[0]) < 1e-9 and abs(rec[1, 0, 6] - gs[1]) < 1e-9
    assert abs(rec[1, 0, 7] - gs[2]) < 1e-10


# ------------------------------------------------------------------ scheduling invariants
def run_state(precision, block, xcd, graphs, ticks=40, buf=1, nt=1):
    y = mc_inputs.draw_y(9, 3)
    ens = mc.Ensemble([mc.Sample(16, 0.05, 100.0, 0.2, True, 2), mc.Sample(32, 0.05, 100.0, 0.2, True, 1),
                       mc.Sample(16, 0.05, 100.0, 0.2, True, 1)], precision)
    ens.init(0, torch.from_numpy(y))
    ens.set_launch(block, xcd, buf, nt)
    ens.use_graphs(graphs)
    ens.step(ticks)
    return [ens.get_state(s).cpu().numpy() for s in range(3)]


@pytest.mark.parametrize("precision", ["f64", "f32s"])
def test_results_do_not_depend_on_launch_shape_or_graphs(precision):
    ref = run_state(precision, 256, 0, False, buf=0, nt=0)
    for block, xcd, graphs, buf, nt in ((128, 1, False, 1, 0), (512, 0, True, 0, 1), (256, 1, True, 1, 1),
                                        (256, 0, False, 1, 0)):
        out = run_state(precision, block, xcd, graphs, buf=buf, nt=nt)
        for a, b in zip(ref, out):
            assert np.array_equal(a, b), (block, xcd, graphs, buf, nt)


def run_rows_state(precision, block, ticks=9):
    """1 x 128^3 (stride 4) + 1 x 256^3: rows of 2 and 4 waves."""
    y = mc_inputs.draw_y(31, 2)
    ens = mc.Ensemble([mc.Sample(128, 0.0125, 1600.0, 0.3, True, 4), mc.Sample(256, 0.00625, 3200.0, 0.3, True, 1)],
                      precision)
    ens.init(0, torch.from_numpy(y))
    ens.set_launch(block, 0, 1, 1)
    ens.use_graphs(False)
    rec = ens.step(ticks - 1, record_every=4).cpu().numpy()
    ens.step(1)
    return [ens.get_state(s).cpu().numpy() for s in range(2)], rec


@pytest.mark.parametrize("precision,blocks", [("f32s", (128, 512, 1024)), ("f64", (128, 256, 512))])
def test_row_exchange_is_bitwise_equal_to_direct_addressing(precision, blocks):
    """Rows longer than a wave held whole by a block move their x-shifted
    populations by lane exchange instead of direct addresses. The arithmetic
    is the same, so the state after several ticks of both AA parities (and
    the fused records) must be bitwise equal: 256^3 with block 128 is
    addressed directly, with larger blocks by exchange (4 waves per row);
    128^3 uses the exchange in every shape."""
    ref, rec_ref = run_rows_state(precision, blocks[0])
    for block in blocks[1:]:
        out, rec = run_rows_state(precision, block)
        for s, (a, b) in enumerate(zip(ref, out)):
            assert np.array_equal(a, b), (block, s)
        # block partials are summed in another order: the records agree to rounding
        assert np.allclose(rec, rec_ref, rtol=1e-12, atol=1e-12), block


def test_checkpoint_restore_is_exact():
    y = mc_inputs.draw_y(4, 2)
    ens = mc.Ensemble([mc.Sample(16, 0.05, 100.0, 0.2, True), mc.Sample(8, 0.05, 100.0, 0.2, True, 2)], "f32s")
    ens.init(0, torch.from_numpy(y))
    ens.step(7)
    ck = ens.checkpoint()
    t0 = ens.ticks
    ens.step(9)
    a = [ens.get_state(s).cpu().numpy() for s in range(2)]
    ens.restore(ck)
    assert ens.ticks == t0
    ens.step(9)
    b = [ens.get_state(s).cpu().numpy() for s in range(2)]
    for x, z in zip(a, b):
        assert np.array_equal(x, z)


def test_instability_flag_names_the_poisoned_sample():
    y = mc_inputs.draw_y(4, 3)
    ens = mc.Ensemble([mc.Sample(16, 0.05, 100.0, 0.2, True)] * 3, "f32s")
    ens.init(0, torch.from_numpy(y))
    ens.step(3)
    ck = ens.checkpoint()
    ens.step(2)
    clean = [ens.get_state(s).cpu().numpy() for s in range(3)]
    ens.restore(ck)
    assert ens.check() == -1
    ens.poison(1, 100, 5)
    ens.step(2)
    assert ens.check() == 1
    with pytest.raises(mc.MclbmError) as ei:
        ens.reduce()
    assert "sample 1" in str(ei.value)
    ens.restore(ck)
    assert ens.check() == -1
    ens.step(2)
    for s in range(3):
        assert np.array_equal(ens.get_state(s).cpu().numpy(), clean[s])


def test_state_errors():
    ens = mc.Ensemble([mc.Sample(8, 0.05, 100.0)], "f64")
    with pytest.raises(mc.MclbmError, match="ERR_STATE"):
        ens.step(1)
    ens.init(0)
    ens.step(0)
    assert ens.ticks == 0
    with pytest.raises(mc.MclbmError, match="ERR_ARG"):
        ens.step(-1)
    with pytest.raises(mc.MclbmError, match="ERR_ARG"):
        ens.moments(3)
    with pytest.raises(mc.MclbmError, match="ERR_UNSUPPORTED"):
        ens.set_launch(1024)


@pytest.mark.parametrize("precision", ["f32s", "f64"])
@pytest.mark.parametrize("q", [27, 19])
def test_degenerate_rest_and_uniform_states(precision, q):
    """Reading C4' (the stabiliser is 2 when <dh|dh> <= 1e-30): a state at
    rest (f = w at every node, g = 0 in the shifted storage) has no
    non-equilibrium part, so it stays exactly at rest on both AA parities,
    with gamma exactly 2 in every record, kinetic energy 0 and mass N^3. A
    uniform flow stays uniform: streaming a uniform field is the identity and
    every node does the same arithmetic, so all nodes stay bitwise equal
    (pin P1 of the oracle, here on the GPU), within rounding of the start,
    and min and max of gamma coincide."""
    n = 16
    smp = mc.Sample(n, 0.05, 100.0, 0.0, False)
    ens = mc.Ensemble([smp, smp], precision, lattice=q)
    ens.init(1)
    _, w = oracle.velocity_set(q)
    U = np.array([0.03, -0.02, 0.01])
    feq = oracle.equilibrium(1.0, U, q)
    for s, f in ((0, w), (1, feq)):
        ens.set_state(s, torch.from_numpy(np.ascontiguousarray(np.repeat(f[:, None], n ** 3, axis=1))).cuda())
    rec = ens.step(7, record_every=1).cpu().numpy()   # 7 ticks: both parities, ending odd
    assert ens.check() == -1
    rest = ens.get_state(0).cpu().numpy().reshape(q, n ** 3)
    assert np.array_equal(rest, np.repeat(w[:, None], n ** 3, axis=1))
    assert np.all(rec[:, 0, 5:8] == 2.0)
    assert np.all(rec[:, 0, 4] == 0.0) and np.all(rec[:, 0, 1:4] == 0.0)
    assert np.all(rec[:, 0, 0] == n ** 3)
    uni = ens.get_state(1).cpu().numpy().reshape(q, n ** 3)
    assert np.array_equal(uni, np.repeat(uni[:, :1], n ** 3, axis=1))
    assert np.all(rec[:, 1, 5] == rec[:, 1, 6])
    # its dh is rounding (FP64: below 1e-30; FP32: within the float
    # threshold): at equilibrium, gamma = 2 in every record
    assert np.all(rec[:, 1, 5:8] == 2.0), rec[:, 1, 5:8]
    # rounding only: FP64, or FP32 storage of g ~ 3e-2 (2e-9 per value; the
    # collision of a rounding-level non-equilibrium part moves it by about as
    # much per step)
    f64 = precision == "f64"
    assert np.max(np.abs(uni[:, 0] - feq)) < (1e-15 if f64 else 1e-7)
    assert np.max(np.abs(rec[:, 1, 0] - n ** 3)) < (1e-9 if f64 else 1e-3)
    mom = rec[:, 1, 1:4] / n ** 3
    assert np.max(np.abs(mom - U)) < (1e-14 if f64 else 1e-7)
    assert np.max(np.abs(rec[:, 1, 4] - 0.5 * np.dot(U, U))) < (1e-15 if f64 else 1e-8)


def test_smallest_lattice_and_set_viscosity():
    """n = 8 (smallest) and a viscosity changed between steps."""
    y = mc_inputs.draw_y(1, 1)
    ens = mc.Ensemble([mc.Sample(8, 0.05, 100.0, 0.3, True)], "f64")
    ens.init(0, torch.from_numpy(y))
    ens.step(5)
    ens.set_viscosity([1 / 50.0])
    ens.step(5)
    _, u_g = gpu_velocity(ens, 0)
    f = oracle.init_populations(8, 0.05, 0.3, y[0], True)
    oracle.run(f, 8, 5, oracle.omega_shear(oracle.lattice_viscosity(8, 0.05, 100.0)))
    oracle.run(f, 8, 5, oracle.omega_shear(oracle.lattice_viscosity(8, 0.05, 50.0)))
    assert rel_l2(u_g, oracle.moments(f, 8)[1]) < 1e-13


def test_stream_copy_kernel():
    src = torch.randn(1 << 20, device="cuda")
    dst = torch.zeros_like(src)
    mc.stream_copy(dst, src)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
