"""GPU parity: the active-set steepest-descent step of eq. 5
(hgl_active_set_step) against the FP64 oracle (oracle.simplex.
active_set_step), and the learning loop with that rule, teacher-forced.

Bar: both sides compute in FP64 and differ only in summation order, so nu,
the direction and the new weights agree to 1e-13 relative to the scale of
g; which weights reach the bound (an integer decision taken from the same
FP64 ratio) must agree exactly on inputs without ties."""
import numpy as np
import pytest

import synth
from oracle import grad as ograd
from oracle import laplacian as lap
from oracle import simplex
from tests.helpers import build, device, hgl, relerr

pytestmark = pytest.mark.gpu


def _case(E, seed, zero_frac):
    rng = synth.rng_for(500 + seed)
    w = rng.dirichlet(np.ones(E) * 0.5)
    w[rng.random(E) < zero_frac] = 0.0
    if not (w > 0).any():
        w[0] = 1.0
    w /= w.sum()
    g = rng.standard_normal(E) / np.sqrt(E)
    return w, g


def _gpu_step(w, g, mu):
    import torch
    dev = device()
    wt = torch.from_numpy(w).to(dev)
    gt = torch.from_numpy(g).to(dev)
    w2, info, d = hgl().active_set_step(wt, gt, mu, direction=True)
    return w2.cpu().numpy(), info, d.cpu().numpy()


@pytest.mark.parametrize("E,seed,zero_frac,mu", [(1, 0, 0.0, 1.0), (7, 1, 0.4, 0.5), (1000, 2, 0.3, 1e-3),
                                                 (1000, 3, 0.6, 10.0), (80_000, 4, 0.3, 1e-5),
                                                 (80_000, 5, 0.5, 100.0), (100_003, 6, 0.05, 1e-4)])
def test_step_against_oracle(E, seed, zero_frac, mu):
    w, g = _case(E, seed, zero_frac)
    w_o, d_o, nu_o, mu_o = simplex.active_set_step(w, g, mu)
    w_g, info, d_g = _gpu_step(w, g, mu)
    scale = np.abs(g).max()
    assert abs(info["nu"] - nu_o) <= 1e-13 * scale
    assert np.abs(d_g - d_o).max() <= 1e-13 * scale
    assert abs(info["mu_eff"] - mu_o) <= 1e-12 * mu_o
    assert np.abs(w_g - w_o).max() <= 1e-13
    assert ((w_g == 0) == (w_o == 0)).all()
    assert (w_g >= 0).all() and abs(w_g.sum() - 1.0) <= 1e-12
    zeros = w == 0
    assert info["released"] == int((zeros & (g < nu_o)).sum())
    assert info["active"] == int((zeros & (g >= nu_o)).sum())


def test_hand_worked_steps():
    w, info, d = _gpu_step(np.array([0.5, 0.5, 0.0]), np.array([1.0, 0.0, 2.0]), 2.0)
    assert w.tolist() == [0.0, 1.0, 0.0] and info["mu_eff"] == 1.0 and info["nu"] == 0.5
    w, info, d = _gpu_step(np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, -1.0]), 1.0)
    assert w.tolist() == [0.5, 0.0, 0.5] and info["nu"] == -0.5
    assert info["released"] == 1 and info["active"] == 1


def test_minimiser_is_a_fixed_point():
    v = synth.rng_for(520).standard_normal(5000) * 0.01
    ws = simplex.project(v)
    _, info, d = _gpu_step(ws, ws - v, 1.0)
    assert np.abs(d).max() <= 1e-15
    assert info["released"] == 0


def test_rejects_bad_input():
    import torch
    from paper_1908_08281_amd._lib import HglError
    dev = device()
    z = torch.zeros(10, dtype=torch.float64, device=dev)
    with pytest.raises(HglError):
        hgl().active_set_step(z, torch.ones_like(z), 1.0)
    with pytest.raises(HglError):
        hgl().active_set_step(torch.full_like(z, 0.1), torch.ones_like(z), 0.0)


def test_learning_loop_active_set_teacher_forced():
    """Each step of the alternating loop with the eq. 5 rule, from the GPU's
    own w_t: the oracle's gradient and active-set step at w_t give the GPU's
    w_{t+1} (teacher forcing), w stays on the simplex, and the objective
    does not increase overall."""
    import torch
    from paper_1908_08281_amd.learn import learn_weights
    dev = device()
    p = synth.weight_learning(N=600, E=480, k=6)
    mu = 0.01
    H = lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx)
    h = build(p, dev)
    Y = torch.from_numpy(p.Y).to(dev, torch.float32)
    w = torch.from_numpy(p.w).to(dev)
    J0 = ograd.objective(H, p.w, p.lam, mu, p.Y)
    eta = None
    for t in range(4):
        w_t = w.cpu().numpy()
        w, recs = learn_weights(h, Y, p.lam, mu, 1, w, eta=eta, tol=3e-7, history=True, rule="active_set")
        eta = recs[0]["eta"]
        g_o = ograd.objective_grad(H, w_t, p.lam, mu, p.Y)
        w_next_o = simplex.active_set_step(w_t, g_o, eta)[0]
        wn = w.cpu().numpy()
        assert relerr(wn, w_next_o) <= 1e-5
        assert (wn >= 0).all() and abs(wn.sum() - 1.0) <= 1e-12
    J4 = ograd.objective(H, w.cpu().numpy(), p.lam, mu, p.Y)
    assert J4 <= J0 * (1 + 1e-9)
