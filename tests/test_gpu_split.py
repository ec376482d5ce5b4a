"""GPU parity of the split sweep, forced on these small systems (below the
automatic threshold): the clean-cell kernel takes the cells of a hole-pair
batch that no other determinant touches, in hole-pair-major order; the
split-correction kernel the batch's other cells; the dense kernel (and the
general kernel for batches it hands over) the remaining batches.  Every
case is checked against the oracle (|A|, fingerprint and selection
bit-exact; E_PT2, S, eps_I within rounding) and against the same call with
the split switched off."""
import numpy as np
import pytest

from gpu_helpers import check_full, run_gpu, e_tolerance
from oracle import oracle as orc
from paper_1902_08154_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1902_08154_amd.api import Context
    c = Context(0)
    yield c
    c.qp_set_split(1)   # QP_SPLIT_AUTO, the default
    c.close()


def _both(ctx, s, E0, n_select):
    ctx.qp_set_split(False)
    u = run_gpu(ctx, s, E0, n_select=n_select)
    ctx.qp_set_split(True)
    g = run_gpu(ctx, s, E0, n_select=n_select)
    return g, u


def _check(ctx, s, n_select, E0=None):
    if E0 is None:
        E0 = orc.energy(s.n_orb, s.h, s.eri, s.dets, s.coefs)
    o = orc.pt2_full(s.n_orb, s.h, s.eri, s.dets, s.coefs, E0, n_select=n_select, eps_gen=True)
    g, u = _both(ctx, s, E0, n_select)
    check_full(g, o, s, n_select)
    check_full(u, o, s, n_select)
    # the same alpha, counts and selection with and without the split
    for key in ("n_alpha", "fingerprint", "n_cells", "n_candidates"):
        if key != "n_candidates":
            assert g["stats"][key] == u["stats"][key], key
    assert np.array_equal(g["sel_dets"], u["sel_dets"])
    rel = [abs(g["e_pt2"][k] - u["e_pt2"][k]) / max(abs(o.e_pt2[k]), 1e-300) for k in range(s.n_states)]
    err = [abs(g["e_pt2"][k] - o.e_pt2[k]) / max(abs(o.e_pt2[k]), 1e-300) for k in range(s.n_states)]
    print(f"{s.name}: |A| = {o.n_alpha}, split vs unsplit rel {max(rel):.2e}, split vs oracle rel {max(err):.2e}, "
          f"handed over {g['stats']['n_alpha_general']}")
    for k in range(s.n_states):
        assert abs(g["e_pt2"][k] - u["e_pt2"][k]) <= 2 * e_tolerance(o, k)
    return g, u, o


def _dets_from_orbitals(n, occs):
    return np.array([synth.det_from_orbitals(n, up, dn) for up, dn in occs])


def test_split_n256_top_orbitals(ctx):
    """n_orb 256 (four words per spin), two states: electrons on orbitals 254
    and 255 and on both sides of every word boundary, so that particles and
    holes reach the last orbital and the 8-bit orbital fields' top value."""
    n = 256
    rng = np.random.default_rng(2560)
    h, eri = synth.make_integrals(rng, n, 8)
    base_up, base_dn = [0, 63, 64, 255], [1, 127, 128, 254]
    occs = {(tuple(base_up), tuple(base_dn))}
    pool = [0, 1, 2, 62, 63, 64, 65, 126, 127, 128, 129, 190, 191, 192, 193, 250, 253, 254, 255]
    while len(occs) < 8:
        up = tuple(sorted(rng.choice(pool, 4, replace=False).tolist()))
        dn = tuple(sorted(rng.choice(pool, 4, replace=False).tolist()))
        occs.add((up, dn))
    occs = sorted(occs)
    dets = _dets_from_orbitals(n, occs)
    c = rng.standard_normal((2, len(occs)))
    c[:, 0] += 3.0
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    s = synth.System("n256_top", 2560, n, 4, 4, h, eri, dets, c)
    _check(ctx, s, n_select=300)


@pytest.mark.parametrize("n,nu,nd,ndet,ns,seed", [(16, 4, 4, 400, 1, 31), (20, 5, 4, 300, 2, 32),
                                                   (12, 3, 3, 250, 3, 33)])
def test_split_dense_connectivity(ctx, n, nu, nd, ndet, ns, seed):
    """Small orbital spaces with many determinants: generators with many
    connected determinants, batches beyond the dense kernel's buffers (handed
    to the general kernel, which then keeps only their flagged cells), and
    batches with integral planes (not split)."""
    s = synth.make_system(f"dense_n{n}", seed, n, nu, nd, ndet, n_states=ns)
    g, _, _ = _check(ctx, s, n_select=200)


@pytest.mark.parametrize("n,nu,nd,ndet,ns", [(48, 6, 6, 300, 1), (96, 4, 4, 150, 2), (130, 3, 3, 200, 2)])
def test_split_grown(ctx, n, nu, nd, ndet, ns):
    """Grown wave functions as in the workloads, 1-3 words per spin."""
    s = synth.make_system(f"grown_n{n}", 7000 + n, n, nu, nd, ndet, n_states=ns)
    _check(ctx, s, n_select=500)


def test_split_generator_list_matches_full(ctx):
    """qp_pt2_generators splits too: a listed generator's eps_I is bit-equal
    to its entry in the full sweep."""
    import torch
    from gpu_helpers import gpu_system
    s = synth.make_system("list", 77, 40, 6, 6, 500, n_states=2)
    E0 = orc.energy(s.n_orb, s.h, s.eri, s.dets, s.coefs)
    dets, coefs = gpu_system(ctx, s)
    E0t = torch.tensor(E0, device=ctx.device)
    full = ctx.pt2(dets, coefs, E0t, eps_gen=True)["eps_gen"].cpu().numpy()
    rng = np.random.default_rng(3)
    gens = rng.choice(s.n_det, 57, replace=False)
    r = ctx.pt2_generators(dets, coefs, E0t, torch.from_numpy(gens.astype(np.int32)))
    assert np.array_equal(r["eps"].cpu().numpy(), full[:, gens])


G_RTOL = 1e-7


def _bwd(ctx, s, E0, gup):
    import torch
    from gpu_helpers import gpu_system
    dets, coefs = gpu_system(ctx, s)
    E0t = torch.tensor(E0, device=ctx.device)
    g = torch.tensor(gup, device=ctx.device)
    gc, gE, gh = ctx.pt2_backward(dets, coefs, E0t, g)
    torch.cuda.synchronize()
    return gc.cpu().numpy(), gE.cpu().numpy(), gh.cpu().numpy()


def _check_bwd(ctx, s):
    E0 = orc.energy(s.n_orb, s.h, s.eri, s.dets, s.coefs)
    gup = np.array([1.0, -0.7, 0.3, 0.5][:s.n_states])
    o = orc.pt2_full(s.n_orb, s.h, s.eri, s.dets, s.coefs, E0, grad_up=gup)
    ctx.qp_set_split(False)
    u = _bwd(ctx, s, E0, gup)
    ctx.qp_set_split(True)
    g = _bwd(ctx, s, E0, gup)
    for name, x, y, ref in zip(("dc", "dE0", "dh"), g, u, (o.dc, o.dE0, o.dh)):
        scale = np.abs(ref).max()
        err, uerr = np.abs(x - ref).max() / scale, np.abs(y - ref).max() / scale
        print(f"{s.name} {name}: split max rel err {err:.2e}, unsplit {uerr:.2e}")
        assert err <= G_RTOL, name
        assert uerr <= G_RTOL, name
    assert np.abs(g[2] - g[2].T).max() <= 1e-12 * np.abs(g[2]).max()


@pytest.mark.parametrize("n,nu,nd,ndet,ns,seed", [(20, 5, 4, 300, 2, 52), (16, 4, 4, 250, 1, 51)])
def test_split_backward_dense_connectivity(ctx, n, nu, nd, ndet, ns, seed):
    """The adjoint of split batches (clean cells: the generator's dc, dE0 and
    dh's diagonal; flagged cells: dc of every connected J and the one-electron
    part of single excitations) against the oracle's gradients."""
    _check_bwd(ctx, synth.make_system(f"bdense_n{n}", seed, n, nu, nd, ndet, n_states=ns))


@pytest.mark.parametrize("n,nu,nd,ndet,ns", [(96, 4, 4, 120, 2), (130, 3, 3, 150, 3)])
def test_split_backward_grown(ctx, n, nu, nd, ndet, ns):
    _check_bwd(ctx, synth.make_system(f"bgrown_n{n}", 7100 + n, n, nu, nd, ndet, n_states=ns))


def test_split_backward_n256_top_orbitals(ctx):
    """Four words per spin, two states, particles and holes on orbitals 254
    and 255."""
    n = 256
    rng = np.random.default_rng(2561)
    h, eri = synth.make_integrals(rng, n, 8)
    occs = {((0, 63, 64, 255), (1, 127, 128, 254))}
    pool = [0, 1, 2, 62, 63, 64, 65, 126, 127, 128, 129, 190, 191, 192, 193, 250, 253, 254, 255]
    while len(occs) < 8:
        up = tuple(sorted(rng.choice(pool, 4, replace=False).tolist()))
        dn = tuple(sorted(rng.choice(pool, 4, replace=False).tolist()))
        occs.add((up, dn))
    occs = sorted(occs)
    dets = _dets_from_orbitals(n, occs)
    c = rng.standard_normal((2, len(occs)))
    c[:, 0] += 3.0
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    _check_bwd(ctx, synth.System("bn256_top", 2561, n, 4, 4, h, eri, dets, c))


def test_fine_filter_count(ctx):
    """stats.n_fine: over every hole batch of every generator, the coarse
    entries J (degree <= 4) lacking at most two of the generator's electrons
    outside the batch's holes, counted here from the determinants: J lacking
    dc electrons reaches all nel + npairs batches when dc <= 2, the 3 single
    batches of its holes and the pairs holding one of them when dc = 3, and
    the 6 pairs inside its holes when dc = 4."""
    s = synth.make_system("fine", 91, 40, 6, 5, 400, n_states=1)
    E0 = orc.energy(s.n_orb, s.h, s.eri, s.dets, s.coefs)
    nel = s.n_up + s.n_dn
    npair = nel * (nel - 1) // 2
    d = s.dets.reshape(s.n_det, -1)
    pc = np.vectorize(lambda x: bin(int(x)).count("1"), otypes=[np.int64])
    want = 0
    for i in range(s.n_det):
        dc = pc(d[i][None, :] & ~d).sum(axis=1)
        for c in dc[dc > 0]:
            if c <= 2:
                want += nel + npair
            elif c == 3:
                want += 3 + npair - (nel - 3) * (nel - 4) // 2
            elif c == 4:
                want += 6
    for split in (True, False):
        ctx.qp_set_split(split)
        g = run_gpu(ctx, s, E0, n_select=0)
        assert g["stats"]["n_fine"] == want, (split, g["stats"]["n_fine"], want)
    ctx.qp_set_split(True)
