"""The package's usage example runs as written and its results hang
together (GPU): the statistics of the records agree with the records, the
last record sits at the tick of the observables (also when they are taken
from the velocity that record tick captured), and the gradient of the
ensemble-mean kinetic energy has the shape of Y."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu
mc = pytest.importorskip("paper_2608_23786_amd")


def test_usage_example():
    samples = [mc.Sample(n=64, u0=0.025, re=1600.0, amp=0.05, project=True)] * 16
    ens = mc.Ensemble(samples, "f32s")
    ens.init(seed=2608)
    ens.autotune()
    rec = ens.step(500, record_every=50)
    assert tuple(rec.shape) == (10, 16, 8)
    s2, ek = ens.observables_range(0, 16)
    assert ens.ticks == 500
    ens.capture_velocity()
    rec_u = ens.step(50, record_every=50)
    s2u, eku = ens.observables_velocity_range(0, 16)
    # the capture is the velocity of tick 500, the state of the observables above
    assert torch.equal(s2u, s2) and torch.equal(eku, ek)
    rec = torch.cat([rec, rec_u])
    ke_mean, ke_std = mc.ensemble_moments(rec[-1, :, 4:5])
    ke = rec[-1, :, 4].cpu().numpy()
    assert abs(float(ke_mean[0]) - ke.mean()) <= 1e-14 * ke.mean()
    assert abs(float(ke_std[0]) - ke.std(ddof=1)) <= 1e-9 * ke.std(ddof=1)
    diss, eta = ens.dissipation(rec, 0, 50)
    assert tuple(diss.shape) == (11, 16) and tuple(eta.shape) == (11,)
    assert torch.all(diss[-1] > 0)
    s2c, ekc = ens.compensate(0, diss[-1], s2, ek)
    assert tuple(s2c.shape) == (16, 32) and tuple(ekc.shape) == (16, 33)
    assert torch.all(torch.isfinite(s2c)) and torch.all(torch.isfinite(ekc))

    y = torch.rand(16, 24, dtype=torch.float64) * 2 - 1
    y.requires_grad_(True)
    J = mc.EnsembleKE.apply(y, mc.Ensemble(samples, "f32s"), 200, 50)
    J.backward()
    assert tuple(y.grad.shape) == (16, 24) and bool(torch.all(torch.isfinite(y.grad)))
    assert np.isfinite(float(J.detach()))
