"""Receptor concentrations and their adjoint on the GPU against the FP64
oracle, on the same seeded inputs and Philox streams.

Tolerances (FP32 kernels vs FP64 oracle):
  * receptor concentrations: relative difference <= 1e-4 on receptors whose
    oracle value is at least 1e-3 of the largest;
  * gradient dL/d(h, q, s_w, v_d): each component within 1e-3 of the oracle's
    (relative), the stated contract of the adjoint;
  * central differences of the GPU forward with common random numbers: within
    3e-2 (kinks of the path -- cell faces, ground folds -- sit at O(delta)
    from some particles, so finite differences are only a rough check).
"""
import os

import numpy as np
import pytest

import oracle
import synth
from parity import log

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0912_3223_amd  # noqa: F401


def stored():
    return synth.load_receptors(os.path.join(HERE, "golden", "c4_receptors.json"))


def loss_weights(c, obs):
    """dL/dc of L = sum (ln(c + eps) - ln(o + eps))^2, eps = 1e-6 max o."""
    eps = 1e-6 * obs.max()
    return 2.0 * (np.log(c + eps) - np.log(obs + eps)) / (c + eps)


def gpu_c_and_grad(case, rec, gbar=None):
    import torch
    import paper_0912_3223_amd as L
    run = L.ReceptorRun(case, rec)
    c = run.forward().cpu().numpy().copy()
    g = None
    if gbar is not None:
        g = run.backward(torch.as_tensor(gbar, dtype=torch.float64)).cpu().numpy().copy()
    return c, g, run


def rel_c(g, o):
    sel = o >= 1e-3 * o.max()
    return float(np.max(np.abs(g - o)[sel] / o[sel]))


def test_receptor_concentration_and_adjoint_match_oracle():
    rec, obs, _ = stored()
    case = synth.c4(n_total=4000, n_steps=1440)
    oc = oracle.Oracle(case)
    oref = oc.receptor_forward(rec)["c"]
    gbar = loss_weights(oref, obs)
    ograd = oc.receptor_adjoint(rec, gbar)
    c, g, _ = gpu_c_and_grad(case, rec, gbar)
    log("receptor c rel %.3e; grad gpu %s oracle %s" % (rel_c(c, oref), g[:4], ograd))
    assert rel_c(c, oref) <= 1e-4
    np.testing.assert_allclose(g[:4], ograd, rtol=1e-3, atol=0)
    # the adjoint's own sum of gbar * c equals the forward's
    assert g[4] == pytest.approx(float(gbar @ c), rel=1e-5)


@pytest.mark.parametrize("kind", ["levels_time_kz2", "vertical_wind_rain_edge"])
def test_adjoint_variants_match_oracle(kind):
    if kind == "levels_time_kz2":
        c = synth.c2(n_total=3000, n_steps=1440, s_release=1440, n_hours=2)
        c = c.with_(physics=synth.replace(c.physics, kz_kind=2))
        lev = (1500.0 * np.linspace(0.0, 1.0, c.field.nz) ** 1.5 + 5.0).astype(np.float32)
        c = synth.with_theta(c.with_(field=synth.replace(c.field, z_levels=lev)), synth.THETA0)
    else:
        c = synth.c4(n_total=3000, n_steps=1440)
        fld = synth.replace(synth.uniform_field(4.0, 0.5, -0.08, bounded=True), x0=-25e3,
                            y0=-25e3, dx=50e3, dy=50e3, dz=1200.0)
        rain = synth.Rain(cx=3000.0, cy=0.0, a=2000.0, b=1500.0, angle=0.3, edge=0.25)
        c = c.with_(field=fld, physics=synth.replace(c.physics, Kh=20.0, kz_kind=0,
                                                     Kz_const=5.0, Lambda0=1e-3, rain=rain))
    rng = np.random.default_rng(7)
    rec = synth.Receptors(tuple(rng.uniform(0.0, 6000.0, 70)), tuple(rng.uniform(-2500, 2500, 70)),
                          tuple(rng.uniform(0.0, 30.0, 70)))
    oc = oracle.Oracle(c)
    oref = oc.receptor_forward(rec)["c"]
    gbar = rng.normal(size=rec.n) / np.maximum(oref, 1e-3 * oref.max())
    ograd = oc.receptor_adjoint(rec, gbar)
    gc, gg, _ = gpu_c_and_grad(c, rec, gbar)
    log("%s: c rel %.3e grad gpu %s oracle %s" % (kind, rel_c(gc, oref), gg[:4], ograd))
    assert rel_c(gc, oref) <= 1e-4
    np.testing.assert_allclose(gg[:4], ograd, rtol=1e-3, atol=0)


def test_full_size_adjoint_on_sampled_particles():
    """The benchmark's 1e6-particle workload: the adjoint of every 997th
    particle id (same Philox counters as the full run) against the oracle's,
    with fixed weights 1/o_r."""
    rec, obs, _ = stored()
    case = synth.c4()
    sub = case.with_(schedule=case.schedule.subset(997, 11))
    gbar = 1.0 / obs
    ograd = oracle.Oracle(sub).receptor_adjoint(rec, gbar)
    oc = oracle.Oracle(sub).receptor_forward(rec)["c"]
    gc, gg, _ = gpu_c_and_grad(sub, rec, gbar)
    log("full-size sampled: c rel %.3e grad gpu %s oracle %s" % (rel_c(gc, oc), gg[:4], ograd))
    assert rel_c(gc, oc) <= 1e-4
    np.testing.assert_allclose(gg[:4], ograd, rtol=1e-3, atol=0)


def test_gradient_against_central_differences_full_size():
    """dL/dtheta of the log misfit at theta0 on the full workload against
    central differences of the GPU forward with common random numbers."""
    import torch
    import paper_0912_3223_amd as L
    rec, obs, _ = stored()
    case = synth.c4()
    run = L.ReceptorRun(case, rec)
    eps = 1e-6 * obs.max()
    o = torch.as_tensor(obs, device="cuda")

    def loss(theta):
        c = run.forward(theta)
        return float(((torch.log(c + eps) - torch.log(o + eps)) ** 2).sum())

    th0 = np.array(synth.THETA0)
    c0 = run.forward(th0).cpu().numpy()
    grad = run.backward(torch.as_tensor(loss_weights(c0, obs))).cpu().numpy()[:4]
    fd = np.zeros(4)
    for j in range(4):
        d = 1e-3 * abs(th0[j])
        tp, tm = th0.copy(), th0.copy()
        tp[j] += d
        tm[j] -= d
        fd[j] = (loss(tp) - loss(tm)) / (2 * d)
    log("full size: adjoint %s central differences %s" % (grad, fd))
    np.testing.assert_allclose(grad, fd, rtol=3e-2)
    # exact: c is proportional to q
    res = np.log(c0 + eps) - np.log(obs + eps)
    assert grad[1] == pytest.approx(2.0 / case.source.q * np.sum(res * c0 / (c0 + eps)), rel=1e-5)


def test_autograd_function_gives_the_adjoint():
    import torch
    import paper_0912_3223_amd as L
    rec, obs, _ = stored()
    case = synth.c4(n_total=20_000, n_steps=720)
    run = L.ReceptorRun(case, rec)
    theta = torch.tensor(synth.THETA0, dtype=torch.float64, requires_grad=True)
    o = torch.as_tensor(obs, device="cuda")
    eps = 1e-6 * float(o.max())
    c = L.ReceptorConcentration.apply(theta, run)
    loss = ((torch.log(c + eps) - torch.log(o + eps)) ** 2).sum()
    loss.backward()
    ref = run.backward(torch.as_tensor(loss_weights(c.detach().cpu().numpy(), obs)))
    np.testing.assert_allclose(theta.grad.numpy(), ref[:4].cpu().numpy(), rtol=1e-12)
    # a second evaluation at another theta reuses the buffers
    c2 = L.ReceptorConcentration.apply(theta.detach() * 1.01, run)
    assert not torch.equal(c2, c)


def test_empty_and_unborn():
    import torch
    import paper_0912_3223_amd as L
    rec, _, _ = stored()
    case = synth.c4(n_total=100, n_steps=120)
    c = case.with_(schedule=synth.replace(case.schedule, n_local=0))
    run = L.ReceptorRun(c, rec)
    assert float(run.forward().abs().sum()) == 0.0
    assert float(run.backward(torch.ones(rec.n, dtype=torch.float64)).abs().sum()) == 0.0
