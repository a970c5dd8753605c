"""GPU parity: weight derivatives through the solve (adjoint CG + edge
contraction), the simplex projection and the autograd binding, against the
FP64 oracle and finite differences (section 2, eq. 4)."""
import numpy as np
import pytest

import synth
from oracle import grad as ograd
from oracle import laplacian as lap
from oracle import simplex, solve
from tests.helpers import build, device, hgl, relerr, say

pytestmark = pytest.mark.gpu


def _small(seed=0, N=900, E=700, k=8):
    p = synth.random_small(seed, N, E, 2, 12, k=k, lam=1.0)
    p.Y = synth.binary_rhs(N, k, 0.05, seed + 5)
    return p


@pytest.mark.parametrize("mode", ["f64", "f32"])
def test_vjp_matches_oracle(mode):
    import torch
    dev = device()
    p = _small()
    H = lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx)
    G = synth.rng_for(3).standard_normal(p.Y.shape)
    g_o, Z_o, F_o = ograd.solve_vjp(H, p.w, p.lam, p.Y, G)
    h = build(p, dev)
    dt = torch.float64 if mode == "f64" else torch.float32
    tol = 1e-12 if mode == "f64" else 3e-7
    F = torch.from_numpy(np.ascontiguousarray(F_o)).to(dev, dt)
    say("vjp", mode)
    g, Z, it, rel, ast = hgl().weight_grad(h, p.lam, F, G=torch.from_numpy(G).to(dev, dt), mode=mode, tol=tol,
                                           want_z=True)
    assert ast == 0
    bound = 1e-10 if mode == "f64" else 1e-5
    assert relerr(g.cpu().numpy(), g_o) <= bound
    assert relerr(Z.cpu().double().numpy(), Z_o) <= (1e-10 if mode == "f64" else 1e-6)


def test_objective_gradient_matches_oracle_and_homogeneity():
    import torch
    dev = device()
    p = _small(1)
    mu = 0.01
    H = lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx)
    h = build(p, dev)
    Y = torch.from_numpy(p.Y).to(dev, torch.float32)
    F, _, _, st = hgl().cg_solve(h, p.lam, Y, tol=3e-7)
    g, _, _, _, ast = hgl().weight_grad(h, p.lam, F, Y=Y, mu=mu, tol=3e-7)
    assert ast == 0
    g = g.cpu().numpy()
    g_o = ograd.objective_grad(H, p.w, p.lam, mu, p.Y, F.cpu().double().numpy())
    assert relerr(g, g_o) <= 1e-5
    # degree-0 homogeneity of A in w: sum_e w_e dJ/dw_e = 2 mu ||w||^2
    lhs = float(p.w @ g)
    assert abs(lhs - 2 * mu * p.w @ p.w) <= 1e-6 * float(np.abs(p.w * g).sum())
    # the adjoint handed back: Z = M^-1 (2 lambda (M F - Y)), same gradient
    g2, Z, _, _, _ = hgl().weight_grad(h, p.lam, F, Y=Y, mu=mu, tol=3e-7, want_z=True)
    assert np.array_equal(g2.cpu().numpy(), g)
    Fd = F.cpu().double().numpy()
    M = lap.system_matrix(H, p.w, p.lam)
    Z_o = solve.solve_dense(M, 2.0 * p.lam * (M @ Fd - p.Y))
    assert relerr(Z.cpu().double().numpy(), Z_o) <= 1e-5


def test_objective_gradient_matches_richardson_fd():
    """64 random edges with w_e > 2h; central differences of the FP64 oracle's
    J at h = 1e-6 with Richardson extrapolation (4 D(h/2) - D(h))/3."""
    import torch
    dev = device()
    p = synth.random_small(4, 300, 240, 2, 10, k=5, lam=1.0)
    p.w = synth.uniform_weights(p.E)
    mu = 0.01
    H = lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx)
    h = build(p, dev)
    Y = torch.from_numpy(p.Y).to(dev)
    F, _, _, _ = hgl().cg_solve(h, p.lam, Y, mode="f64", tol=1e-13)
    g, _, _, _, ast = hgl().weight_grad(h, p.lam, F, Y=Y, mu=mu, mode="f64", tol=1e-13)
    assert ast == 0
    g = g.cpu().numpy()
    edges = synth.rng_for(9).choice(np.nonzero(p.w > 2e-6)[0], size=64, replace=False)
    J = lambda w: ograd.objective(H, w, p.lam, mu, p.Y)  # noqa: E731
    fd = np.array([ograd.richardson_difference(J, p.w, int(e), 1e-6) for e in edges])
    assert np.linalg.norm(g[edges] - fd) / np.linalg.norm(fd) <= 1e-5


def test_simplex_projection_matches_oracle():
    import torch
    dev = device()
    for seed, E in [(0, 1), (1, 7), (2, 1000), (3, 80_000)]:
        v = synth.rng_for(seed).normal(1.0 / E, 3.0 / E, size=E)
        w = hgl().project_simplex(torch.from_numpy(v).to(dev)).cpu().numpy()
        ref = simplex.project(v)
        assert np.allclose(w, ref, rtol=0, atol=1e-15 + 1e-13 * ref.max())
        assert np.all(w >= 0) and abs(w.sum() - 1) < 1e-12
    w0 = synth.dirichlet_weights(500, 4)
    assert np.allclose(hgl().project_simplex(torch.from_numpy(w0).to(dev)).cpu().numpy(), w0, atol=1e-15)


def test_projected_gradient_step_matches_oracle():
    """hgl_projected_gradient_step against the oracle's step rule and
    projection: a given eta, and eta set from the gradient (reported on the
    device); sizes from one entry to the learning workload's E."""
    import torch
    dev = device()
    for seed, E in [(0, 1), (1, 7), (2, 1000), (3, 80_000)]:
        say("pg step", E)
        w = synth.dirichlet_weights(E, seed)
        g = synth.rng_for(seed + 10).normal(0.0, 1.0, size=E)
        wd, gd = torch.from_numpy(w).to(dev), torch.from_numpy(g).to(dev)
        eta_o = simplex.initial_step(w, g)
        w1, e1 = hgl().projected_gradient_step(wd, gd, None)
        eta1 = float(e1.item())
        assert abs(eta1 - eta_o) <= 1e-14 * abs(eta_o)
        ref = simplex.project(w - eta1 * g)
        assert np.allclose(w1.cpu().numpy(), ref, rtol=0, atol=1e-15 + 1e-13 * ref.max())
        w2, e2 = hgl().projected_gradient_step(wd, gd, 0.37 / E)
        assert float(e2.item()) == 0.37 / E
        ref2 = simplex.project(w - (0.37 / E) * g)
        assert np.allclose(w2.cpu().numpy(), ref2, rtol=0, atol=1e-15 + 1e-13 * ref2.max())
        assert abs(float(w2.sum()) - 1.0) < 1e-12 and bool((w2 >= 0).all())
    from paper_1908_08281_amd import _lib
    with pytest.raises(_lib.HglError):
        hgl().projected_gradient_step(wd, gd, float("nan"))


def test_autograd_function():
    import torch
    from paper_1908_08281_amd.learn import HypergraphSolve
    dev = device()
    p = _small(2, N=500, E=400, k=4)
    h = build(p, dev)
    w = torch.from_numpy(p.w).to(dev).requires_grad_(True)
    Y = torch.from_numpy(p.Y).to(dev, torch.float64).requires_grad_(True)
    C = torch.from_numpy(synth.rng_for(7).standard_normal(p.Y.shape)).to(dev)
    F = HypergraphSolve.apply(w, Y, h, p.lam, 1e-13, "f64")
    loss = (F * C).sum()
    loss.backward()
    H = lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx)
    g_o, Z_o, _ = ograd.solve_vjp(H, p.w, p.lam, p.Y, C.cpu().numpy())
    assert relerr(w.grad.cpu().numpy(), g_o) <= 1e-9
    assert relerr(Y.grad.cpu().numpy(), Z_o) <= 1e-9


def test_learning_loop_teacher_forced():
    """Each projected-gradient step from the GPU's own w_t: the oracle's
    gradient and projected step at w_t agree (teacher forcing), and the
    objective does not increase overall."""
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
        w, recs = learn_weights(h, Y, p.lam, mu, 1, w, eta=eta, tol=3e-7, history=True)
        assert recs[0]["cg_status"] == 0 and recs[0]["adjoint_status"] == 0
        g_o = ograd.objective_grad(H, w_t, p.lam, mu, p.Y)
        if eta is None:  # the library's step from the first gradient
            assert abs(recs[0]["eta"] - simplex.initial_step(w_t, g_o)) <= 1e-4 * recs[0]["eta"]
        eta = recs[0]["eta"]
        w_next_o = simplex.project(w_t - eta * g_o)
        assert relerr(w.cpu().numpy(), w_next_o) <= 1e-5
    J4 = ograd.objective(H, w.cpu().numpy(), p.lam, mu, p.Y)
    assert J4 <= J0 * (1 + 1e-9)


@pytest.mark.slow
def test_full_size_gradient_against_sparse_oracle():
    """Differentiation workload at full N (100,000 vertices, 80,000 hyperedges)
    on 16 of the tag columns: every edge's gradient against the sparse FP64
    oracle, and homogeneity."""
    import torch
    dev = device()
    p = synth.weight_learning(k=16)
    mu = 0.01
    h = build(p, dev)
    Y = torch.from_numpy(p.Y).to(dev, torch.float32)
    say("grad full size")
    F, _, _, st = hgl().cg_solve(h, p.lam, Y, tol=5e-7)
    g, _, _, _, ast = hgl().weight_grad(h, p.lam, F, Y=Y, mu=mu, tol=5e-7)
    assert ast == 0
    g = g.cpu().numpy()
    op = lap.SparseOperator(p.N, p.E, p.edge_ptr, p.edge_vtx, p.w, p.lam)
    g_o = ograd.objective_grad_sparse(op, p.w, p.lam, mu, p.Y, F.cpu().double().numpy())
    assert relerr(g, g_o) <= 1e-5
    assert abs(p.w @ g - 2 * mu * p.w @ p.w) <= 1e-6 * float(np.abs(p.w * g).sum())


@pytest.mark.slow
def test_full_size_gradient_against_richardson_fd():
    """The differentiation workload's graph at full size (N = 100,000,
    E = 80,000, w = 1/E, lambda = 1, mu = 0.01) on two tag columns: the
    adjoint gradient of the FP32 solve on 64 random edges with w_e > 2h
    against central differences of the FP64 objective at h = 1e-6 with
    Richardson extrapolation (reading R14: plain h = 1e-6 differences carry
    an O((h/delta_v)^2) error at this weight scale), computed on every host
    core by the sparse oracle."""
    import torch
    from tests import fd_pool
    dev = device()
    p = synth.weight_learning(k=2)
    mu, h_fd = 0.01, 1e-6
    h = build(p, dev)
    Y = torch.from_numpy(p.Y).to(dev, torch.float32)
    say("grad full size vs fd")
    F, _, rel, st = hgl().cg_solve(h, p.lam, Y, tol=1e-7)
    assert st == 0
    g, _, _, _, ast = hgl().weight_grad(h, p.lam, F, Y=Y, mu=mu, tol=1e-7)
    assert ast == 0
    g = g.cpu().numpy()
    edges = synth.rng_for(19).choice(np.nonzero(p.w > 2 * h_fd)[0], size=64, replace=False)
    fd = fd_pool.richardson_gradient(p, mu, edges, h_fd)
    assert np.linalg.norm(g[edges] - fd) / np.linalg.norm(fd) <= 1e-5


@pytest.mark.slow
def test_full_size_gradient_k500_homogeneity_and_additivity():
    """The differentiation workload as the bench runs it (N=100,000,
    E=80,000, all 500 tag columns; FP32 solve and adjoint to relres 5e-7).
    The FP64 oracle needs minutes at k=500, so the full launch is pinned by
    properties that hold at any size: homogeneity (sum_e w_e dL/dw_e =
    2 mu |w|^2, A being degree-0 homogeneous in w) and additivity over the
    columns (the loss is a sum over columns, so the gradient of all 500 is
    the sum of the gradients of two halves, each its own launch, minus one
    2 mu w).  The 16-column launch is checked against the oracle above."""
    import torch
    dev = device()
    p = synth.weight_learning()
    mu = 0.01
    tol = 1e-6 / (1 + 1 / p.lam)
    h = build(p, dev)
    Y = torch.from_numpy(p.Y).to(dev, torch.float32)
    say("grad full size k=500")
    F, _, rel, st = hgl().cg_solve(h, p.lam, Y, tol=tol)
    assert st == 0 and np.all(rel <= tol)
    g, _, _, _, ast = hgl().weight_grad(h, p.lam, F, Y=Y, mu=mu, tol=tol)
    assert ast == 0
    g = g.cpu().numpy()
    assert abs(p.w @ g - 2 * mu * p.w @ p.w) <= 1e-6 * float(np.abs(p.w * g).sum())
    halves = []
    for c0, c1 in ((0, 250), (250, 500)):
        gh, _, _, _, _ = hgl().weight_grad(h, p.lam, F[:, c0:c1].contiguous(), Y=Y[:, c0:c1].contiguous(), mu=mu,
                                        tol=tol)
        halves.append(gh.cpu().numpy() - 2 * mu * p.w)
    assert relerr(g - 2 * mu * p.w, halves[0] + halves[1]) <= 1e-6

