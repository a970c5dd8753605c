"""GPU parity: the power-scheme sketch of eq. 10 (Y = (A A')^q A Omega by
2q+1 products with no orthonormalisation in between, one CholQR2 at the end)
in place of Algorithm 1's steps 2-3, against the oracle's power scheme on the
same sketch Omega."""
import ctypes as C

import numpy as np
import pytest

import synth
from oracle import laplacian as lap
from oracle import rsvd, solve
from tests.helpers import build, colrelerr, device, hgl, say

pytestmark = pytest.mark.gpu


def _bits(p, l, seed):
    return synth.gaussian_sketch(p.N, l, seed)


def _dev_bits(bits, dev):
    import torch
    return torch.from_numpy(bits.view(np.int16).copy()).to(dev)


def _problem():
    return synth.tessellated(n_blocks=6, lo=150, hi=300, k_rhs=12)


def _blocks(p):
    A = lap.adjacency(lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx), p.w)
    return rsvd.tessellate(A, p.blocks)


@pytest.mark.parametrize("q", [1, 2])
def test_power_f64_matches_oracle(q):
    """FP64 products: top-k sigma and the approximation error of the power
    scheme agree with the oracle's power scheme on the same Omega."""
    dev = device()
    p = _problem()
    k, pp = 24, 8
    bits, vals = _bits(p, k + pp, 19)
    say("rsvd power f64 q", q)
    h = build(p, dev)
    U, sig = hgl().block_rsvd(h, p.blocks, k, pp, q, sketch="f64", omega=_dev_bits(bits, dev), scheme="power")
    U, sig = U.cpu().double().numpy(), sig.cpu().numpy()
    for b, Ab in enumerate(_blocks(p)):
        o0, o1 = p.blocks[b], p.blocks[b + 1]
        Uo, so, _ = rsvd.randomized_svd_power(Ab, vals[o0:o1], q)
        assert np.max(np.abs(sig[b] - so[:k]) / so[:k]) <= 1e-9
        Ub = U[o0:o1]
        err_gpu = np.linalg.norm(Ab - Ub @ np.diag(sig[b]) @ Ub.T)
        err_or = np.linalg.norm(Ab - Uo[:, :k] @ np.diag(so[:k]) @ Uo[:, :k].T)
        assert abs(err_gpu - err_or) <= 1e-6 * err_or   # U is stored in FP32


def test_power_bf16_matches_oracle():
    """BF16 blocks and sketch, FP32 products: against the oracle's power scheme
    on the BF16-rounded blocks (the operands between products carry about 16
    bits, so the bar is that of the BF16 Algorithm 1)."""
    dev = device()
    p = _problem()
    k, pp, q = 24, 8, 2
    bits, vals = _bits(p, k + pp, 23)
    say("rsvd power bf16")
    h = build(p, dev)
    U, sig = hgl().block_rsvd(h, p.blocks, k, pp, q, sketch="bf16", omega=_dev_bits(bits, dev), scheme="power")
    U, sig = U.cpu().double().numpy(), sig.cpu().numpy()
    for b, Ab in enumerate(_blocks(p)):
        o0, o1 = p.blocks[b], p.blocks[b + 1]
        Ab16 = synth.bf16_round(Ab)[1]
        Uo, so, _ = rsvd.randomized_svd_power(Ab16, vals[o0:o1], q)
        assert np.max(np.abs(sig[b] - so[:k]) / so[:k]) <= 1e-3
        Ub = U[o0:o1]
        err_gpu = np.linalg.norm(Ab - Ub @ np.diag(sig[b]) @ Ub.T)
        err_or = np.linalg.norm(Ab - Uo[:, :k] @ np.diag(so[:k]) @ Uo[:, :k].T)
        assert abs(err_gpu - err_or) <= 1e-3 * err_or


@pytest.mark.parametrize("sketch", ["bf16", "f64"])
def test_q0_schemes_identical(sketch):
    """With q = 0 both schemes are one product and one CholQR2: bitwise equal."""
    dev = device()
    p = _problem()
    bits, _ = _bits(p, 20, 29)
    h = build(p, dev)
    om = _dev_bits(bits, dev)
    U1, s1 = hgl().block_rsvd(h, p.blocks, 16, 4, 0, sketch=sketch, omega=om, scheme="subspace")
    U2, s2 = hgl().block_rsvd(h, p.blocks, 16, 4, 0, sketch=sketch, omega=om, scheme="power")
    assert np.array_equal(U1.cpu().numpy(), U2.cpu().numpy())
    assert np.array_equal(s1.cpu().numpy(), s2.cpu().numpy())


def test_power_refined_solve_matches_cholesky():
    """The block inverse from the power scheme, refined by PCG to 1e-6."""
    import torch
    dev = device()
    p = _problem()
    h = build(p, dev)
    Y = torch.from_numpy(p.Y).to(dev, torch.float32)
    tol = 1e-6 / (1 + 1 / p.lam)
    F, it, rel, sig, st = hgl().block_rsvd_invert(h, p.lam, p.blocks, Y, 24, 8, 2, seed=3, refine_tol=tol,
                                                  scheme="power")
    assert st == 0 and np.all(rel <= tol)
    H = lap.incidence_dense(p.N, p.E, p.edge_ptr, p.edge_vtx)
    Fo = solve.solve_dense(lap.system_matrix(H, p.w, p.lam), p.Y)
    assert colrelerr(F.cpu().numpy(), Fo).max() <= 1e-6


def test_unknown_scheme_rejected():
    import torch
    from paper_1908_08281_amd import _lib
    dev = device()
    p = _problem()
    h = build(p, dev)
    off = np.ascontiguousarray(p.blocks, dtype=np.int32)
    U = torch.empty((p.N, 8), dtype=torch.float32, device=dev)
    opts = _lib.RsvdOpts(8, 4, 1, _lib.HGL_SKETCH_BF16, 1, 1e-6, 10, 0, 7)
    lib = _lib.load()
    with torch.cuda.device(dev):
        st = lib.hgl_block_rsvd(h.ptr, len(off) - 1, off.ctypes.data_as(_lib.I32P), C.byref(opts),
                                C.c_void_p(0), C.c_void_p(U.data_ptr()), C.c_void_p(0),
                                C.c_void_p(torch.cuda.current_stream(dev).cuda_stream))
    assert st == _lib.HGL_EINVAL
    assert "scheme" in lib.hgl_last_error().decode()
