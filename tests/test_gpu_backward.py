"""GPU adjoint: dE_PT2/dc, dE_PT2/dE0 and dE_PT2/dh from the backward sweep
against the oracle's analytic gradients (themselves pinned by finite
differences) and against finite differences of the GPU forward sweep.
Tolerance: 1e-7 relative to the largest gradient component."""
import numpy as np
import pytest

from gpu_helpers import gpu_system
from oracle import oracle as orc
from paper_1902_08154_amd import synth

pytestmark = pytest.mark.gpu

G_RTOL = 1e-7


@pytest.fixture(scope="module")
def ctx():
    from paper_1902_08154_amd.api import Context
    c = Context(0)
    yield c
    c.close()


CASES = [
    ("b_n20_3a3b", 20, 3, 3, 50, 2),
    ("b_n40_5a3b_open", 40, 5, 3, 30, 1),
    ("b_n70_3a2b_nint2", 70, 3, 2, 20, 3),
    ("b_n130_2a2b_nint3", 130, 2, 2, 12, 1),
]


def _grads(ctx, s, E0, gup):
    import torch
    dets, coefs = gpu_system(ctx, s)
    E0t = torch.tensor(E0, device=ctx.device)
    g = torch.tensor(gup, device=ctx.device)
    gc, gE, gh = ctx.pt2_backward(dets, coefs, E0t, g)
    torch.cuda.synchronize()
    return gc.cpu().numpy(), gE.cpu().numpy(), gh.cpu().numpy()


@pytest.mark.parametrize("name,n,nu,nd,ndet,ns", CASES)
def test_backward_vs_oracle(ctx, name, n, nu, nd, ndet, ns):
    s = synth.make_system(name, 808 + n + ndet, n, nu, nd, ndet, n_states=ns)
    E0 = orc.energy(n, s.h, s.eri, s.dets, s.coefs)
    gup = np.array([1.0, -0.7, 0.3, 0.5][:ns])
    o = orc.pt2_full(n, s.h, s.eri, s.dets, s.coefs, E0, grad_up=gup)
    gc, gE, gh = _grads(ctx, s, E0, gup)
    assert np.abs(gc - o.dc).max() <= G_RTOL * np.abs(o.dc).max()
    assert np.allclose(gE, o.dE0, rtol=G_RTOL, atol=0)
    assert np.abs(gh - o.dh).max() <= G_RTOL * np.abs(o.dh).max()
    assert np.abs(gh - gh.T).max() <= 1e-12 * np.abs(gh).max()


def test_backward_finite_differences_of_gpu_forward(ctx):
    """E is quadratic in c at fixed E0, so central differences of the GPU
    forward sweep are exact up to rounding."""
    import torch
    from paper_1902_08154_amd.api import to_device_dets
    s = synth.make_system("fd", 99, 24, 4, 4, 40, n_states=1)
    E0 = orc.energy(s.n_orb, s.h, s.eri, s.dets, s.coefs)
    gc, gE, gh = _grads(ctx, s, E0, [1.0])
    dev = ctx.device
    dets = to_device_dets(s.dets, dev)
    E0t = torch.tensor(E0, device=dev)

    def energy(c):
        return float(ctx.pt2(dets, torch.from_numpy(c).to(dev), E0t)["e_pt2"].item())

    rng = np.random.default_rng(1)
    for j in rng.choice(s.n_det, 6, replace=False):
        eps = 1e-3
        cp = s.coefs.copy(); cp[0, j] += eps
        cm = s.coefs.copy(); cm[0, j] -= eps
        fd = (energy(cp) - energy(cm)) / (2 * eps)
        assert abs(fd - gc[0, j]) <= 1e-7 * max(1.0, np.abs(gc).max())
    # Euler identity: sum_J c_J dE/dc_J = 2 E
    e = energy(s.coefs.copy())
    assert abs(float(s.coefs[0] @ gc[0]) - 2 * e) <= 1e-9 * max(1.0, abs(e))


def test_autograd_function_matches_oracle(ctx):
    """PT2Function: torch.autograd through the HIP forward and adjoint sweeps,
    for a weighted sum of the states' E_PT2, against the oracle's gradients."""
    import torch
    from paper_1902_08154_amd.api import pt2_autograd, to_device_dets
    s = synth.make_system("ag_n24_4a3b", 4242, 24, 4, 3, 40, n_states=2)
    E0 = orc.energy(s.n_orb, s.h, s.eri, s.dets, s.coefs)
    w = np.array([0.8, -1.3])
    o = orc.pt2_full(s.n_orb, s.h, s.eri, s.dets, s.coefs, E0, grad_up=w)
    dev = ctx.device
    dets = to_device_dets(s.dets, dev)
    coefs = torch.tensor(s.coefs, device=dev, requires_grad=True)
    E0t = torch.tensor(E0, device=dev, requires_grad=True)
    h = torch.tensor(s.h, device=dev, requires_grad=True)
    eri = torch.tensor(s.eri, device=dev)
    e = pt2_autograd(ctx, dets, coefs, E0t, h, eri)
    loss = (e * torch.tensor(w, device=dev)).sum()
    gc, gE, gh = torch.autograd.grad(loss, (coefs, E0t, h))
    torch.cuda.synchronize()
    gc, gE, gh = gc.cpu().numpy(), gE.cpu().numpy(), gh.cpu().numpy()
    assert np.allclose(e.detach().cpu().numpy(), o.e_pt2, rtol=1e-9, atol=0)
    assert np.abs(gc - o.dc).max() <= G_RTOL * np.abs(o.dc).max()
    assert np.allclose(gE, o.dE0, rtol=G_RTOL, atol=0)
    assert np.abs(gh - o.dh).max() <= G_RTOL * np.abs(o.dh).max()
    # only the requested gradient: E0 alone
    E0b = torch.tensor(E0, device=dev, requires_grad=True)
    (gE2,) = torch.autograd.grad((pt2_autograd(ctx, dets, coefs.detach(), E0b, h.detach(), eri) *
                                  torch.tensor(w, device=dev)).sum(), (E0b,))
    assert np.allclose(gE2.cpu().numpy(), o.dE0, rtol=G_RTOL, atol=0)
