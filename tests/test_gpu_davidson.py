"""GPU parity of the Davidson sigma-build and diagonaliser (sec. "Davidson
diagonalization"): W = H U and W = S^2 U against the oracle's dense matrices,
eigenpairs against a dense symmetric eigensolver of the oracle's H, and at
the c2 size the Rayleigh quotient of the returned vector recomputed by the
oracle."""
import numpy as np
import pytest

from gpu_helpers import gpu_system
from oracle import oracle as orc
from oracle import sq_tier0 as sq
from paper_1902_08154_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1902_08154_amd.api import Context
    c = Context(0)
    yield c
    c.close()


SYS = [("d_n24_4a4b", 24, 4, 4, 300, 4), ("d_n70_3a2b_nint2", 70, 3, 2, 120, 3), ("d_n40_5a3b", 40, 5, 3, 200, 2)]


@pytest.mark.parametrize("name,n,nu,nd,ndet,nv", SYS)
def test_sigma_matches_dense_matrices(ctx, name, n, nu, nd, ndet, nv):
    import torch
    s = synth.make_system(name, 3030 + n, n, nu, nd, ndet)
    dets, _ = gpu_system(ctx, s)
    U = np.random.default_rng(n).standard_normal((nv, ndet))
    W = ctx.sigma(dets, torch.from_numpy(U)).cpu().numpy()
    H = orc.hamiltonian(n, s.h, s.eri, s.dets)
    ref = U @ H.T
    assert np.abs(W - ref).max() <= 1e-12 * np.abs(H).max() * np.abs(U).sum(axis=1).max()
    W2 = ctx.sigma(dets, torch.from_numpy(U), s2=True).cpu().numpy()
    S2 = orc.s2_matrix(n, s.dets)
    assert np.abs(W2 - U @ S2.T).max() <= 1e-12 * np.abs(U).sum(axis=1).max()


def test_sigma_reuse(ctx):
    """QP_SIGMA_REUSE gives the same bits as a fresh preparation, and a change
    of integrals or of the determinant list prepares again."""
    import torch
    s = synth.make_system("d_n24_4a4b", 3054, 24, 4, 4, 300)
    dets, _ = gpu_system(ctx, s)
    U = torch.from_numpy(np.random.default_rng(5).standard_normal((3, 300)))
    W0 = ctx.sigma(dets, U).cpu().numpy()
    W1 = ctx.sigma(dets, U, reuse=True).cpu().numpy()
    W2 = ctx.sigma(dets, U, s2=True, reuse=True).cpu().numpy()
    assert np.array_equal(W0, W1)
    assert np.abs(W2 - U.numpy() @ orc.s2_matrix(24, s.dets).T).max() <= 1e-12 * np.abs(U.numpy()).sum(axis=1).max()
    # other integrals at the same n_orb: the reuse flag must not keep the old diagonal
    t = synth.make_system("d_n24_4a4b_b", 3055, 24, 4, 4, 300)
    ctx.qp_set_integrals(torch.from_numpy(t.h).to(ctx.device), torch.from_numpy(t.eri).to(ctx.device))
    W3 = ctx.sigma(dets, U, reuse=True).cpu().numpy()
    H = orc.hamiltonian(24, t.h, t.eri, s.dets)
    assert np.abs(W3 - U.numpy() @ H.T).max() <= 1e-12 * np.abs(H).max() * np.abs(U.numpy()).sum(axis=1).max()
    # a shorter list at a new address
    d2, _ = gpu_system(ctx, synth.make_system("d_n24_4a4b_c", 3056, 24, 4, 4, 120))
    W4 = ctx.sigma(d2, U[:, :120].contiguous(), reuse=True).cpu().numpy()
    W5 = ctx.sigma(d2, U[:, :120].contiguous()).cpu().numpy()
    assert np.array_equal(W4, W5)


def test_davidson_full_space_matches_dense_eigensolver(ctx):
    """The whole FCI space of n=6, 2+2 electrons: exact eigenpairs."""
    import torch
    from paper_1902_08154_amd.api import to_device_dets
    n, nup, ndn = 6, 2, 2
    rng = np.random.default_rng(8)
    h, eri = synth.make_integrals(rng, n, 12)
    basis = sq.fci_space(n, nup, ndn)
    dets_np = np.array([sq.to_words(d, n) for d in basis])
    dev = ctx.device
    ctx.qp_set_integrals(torch.from_numpy(h).to(dev), torch.from_numpy(eri).to(dev))
    dets = to_device_dets(dets_np, dev)
    r = ctx.davidson(dets, n_states=3, tol=1e-9)
    H = orc.hamiltonian(n, h, eri, dets_np)
    ev, vec = np.linalg.eigh(H)
    assert np.allclose(r["E"], ev[:3], rtol=0, atol=1e-10 * max(1.0, abs(ev[0])))
    C = r["C"].cpu().numpy()
    for k in range(3):
        res = H @ C[k] - r["E"][k] * C[k]
        assert np.linalg.norm(res) < 1e-8 and abs(np.linalg.norm(C[k]) - 1) < 1e-12
    S2 = orc.s2_matrix(n, dets_np)
    assert np.allclose(r["s2"], [C[k] @ S2 @ C[k] for k in range(3)], atol=1e-9)


@pytest.mark.parametrize("name,n,nu,nd,ndet,nv", SYS[:2])
def test_davidson_on_selected_spaces(ctx, name, n, nu, nd, ndet, nv):
    s = synth.make_system(name, 4040 + n, n, nu, nd, ndet)
    dets, _ = gpu_system(ctx, s)
    ns = 2
    r = ctx.davidson(dets, n_states=ns, tol=1e-9)
    H = orc.hamiltonian(n, s.h, s.eri, s.dets)
    ev = np.linalg.eigvalsh(H)
    assert np.allclose(r["E"], ev[:ns], rtol=0, atol=1e-10 * max(1.0, abs(ev[0])))


def test_davidson_c2_prefix_against_dense_eigensolver(ctx):
    """The first 2,000 determinants of the c2 wave function (n_orb 64, 10+10):
    the two lowest eigenvalues of the dense H."""
    s = synth.workload(2, n_det=2000)
    dets, _ = gpu_system(ctx, s)
    r = ctx.davidson(dets, n_states=2, tol=1e-8, max_iter=400)
    ev = np.linalg.eigvalsh(orc.hamiltonian(s.n_orb, s.h, s.eri, s.dets))
    print("davidson c2 prefix", r["E"], ev[:2], r["n_iter"], flush=True)
    assert np.allclose(r["E"], ev[:2], rtol=1e-11, atol=0)


def test_davidson_c2_full_size(ctx):
    """The c2 determinant space (10^4), started from the wave function's own
    coefficients: the eigenvalue equals the oracle's Rayleigh quotient
    <C|H|C>/<C|C> of the returned vector, and the residual recomputed with a
    separate sigma-build is below the tolerance."""
    import torch
    s = synth.workload(2)
    dets, coefs = gpu_system(ctx, s)
    r = ctx.davidson(dets, n_states=1, guess=coefs, tol=1e-8, max_iter=400)
    C = r["C"].cpu().numpy()
    print("davidson c2", r["E"], r["n_iter"], flush=True)
    E = orc.energy(s.n_orb, s.h, s.eri, s.dets, C)
    assert abs(E[0] - r["E"][0]) <= 1e-10 * abs(E[0])
    W = ctx.sigma(dets, r["C"]).cpu().numpy()
    assert np.linalg.norm(W[0] - r["E"][0] * C[0]) < 1e-8
    assert r["E"][0] <= float(orc.energy(s.n_orb, s.h, s.eri, s.dets, s.coefs)[0])
