"""GPU parity: the HIP sweep (through the C ABI) against the CPU oracle on the
same seeded inputs.  Bit-exact: |A|, the alpha-set fingerprint, the selected
bit strings.  FP64 within a relative 1e-10: E_PT2, S, eps_I, selected e."""
import numpy as np
import pytest

from gpu_helpers import compare_full, run_gpu, E_RTOL
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


def _E0(s):
    return orc.energy(s.n_orb, s.h, s.eri, s.dets, s.coefs)


def test_c1_full_alpha_dump(ctx):
    """n=12, 3+3 electrons, 50 dets: every alpha, in selection order."""
    s = synth.workload(1)
    E0 = _E0(s)
    o = orc.pt2_full(s.n_orb, s.h, s.eri, s.dets, s.coefs, E0, n_select=10 ** 6, eps_gen=True)
    compare_full(ctx, s, E0, n_select=o.n_alpha + 7)


MID = [
    # (name, n_orb, n_up, n_dn, n_det, n_states)  several slabs, ragged tails
    ("n24_4a4b", 24, 4, 4, 60, 2),
    ("n40_5a3b_open", 40, 5, 3, 40, 1),
    ("n70_3a2b_nint2", 70, 3, 2, 25, 3),
    ("n130_2a2b_nint3", 130, 2, 2, 20, 1),
    ("n200_2a1b_nint4", 200, 2, 1, 10, 2),
    ("n64_4a4b_4states", 64, 4, 4, 12, 4),
]


@pytest.mark.parametrize("name,n,nu,nd,ndet,ns", MID)
def test_mid_systems(ctx, name, n, nu, nd, ndet, ns):
    s = synth.make_system(name, 4242 + n + ndet, n, nu, nd, ndet, n_states=ns)
    E0 = _E0(s)
    compare_full(ctx, s, E0, n_select=150)


def test_single_determinant(ctx):
    s = synth.make_system("single", 5, 16, 3, 3, 1)
    E0 = _E0(s) - 0.25
    compare_full(ctx, s, E0, n_select=50)


def test_full_space_has_no_alpha(ctx):
    n, nu, nd = 6, 2, 2
    rng = np.random.default_rng(3)
    h, eri = synth.make_integrals(rng, n, 12)
    basis = sq.fci_space(n, nu, nd)
    dets = np.array([sq.to_words(d, n) for d in basis])
    c = rng.standard_normal((1, len(basis)))
    s = synth.System("fci", 3, n, nu, nd, h, eri, dets, c)
    g = run_gpu(ctx, s, [-1.0], n_select=10)
    assert g["stats"]["n_alpha"] == 0
    assert g["e_pt2"][0] == 0.0
    assert g["sel_dets"].shape[0] == 0


def test_select_more_than_alpha(ctx):
    s = synth.make_system("small", 9, 8, 2, 2, 6)
    E0 = _E0(s)
    g, o = compare_full(ctx, s, E0, n_select=100000)
    assert g["sel_dets"].shape[0] == o.n_alpha


def test_energy_matches_oracle(ctx):
    import torch
    from gpu_helpers import gpu_system
    for (name, n, nu, nd, ndet, ns) in MID[:4]:
        s = synth.make_system(name, 4242 + n + ndet, n, nu, nd, ndet, n_states=ns)
        dets, coefs = gpu_system(ctx, s)
        e = ctx.energy(dets, coefs).cpu().numpy()
        assert np.allclose(e, _E0(s), rtol=1e-12, atol=1e-12)


def test_determinism(ctx):
    s = synth.make_system("det", 77, 32, 4, 4, 80, n_states=2)
    E0 = _E0(s)
    a = run_gpu(ctx, s, E0, n_select=300)
    b = run_gpu(ctx, s, E0, n_select=300)
    assert np.array_equal(a["e_pt2"], b["e_pt2"])
    assert np.array_equal(a["eps_gen"], b["eps_gen"])
    assert np.array_equal(a["sel_dets"], b["sel_dets"])


def test_error_codes(ctx):
    import torch
    from paper_1902_08154_amd.api import QPError, Context, to_device_dets
    from paper_1902_08154_amd import _lib
    s = synth.make_system("err", 11, 10, 2, 2, 8)
    dev = ctx.device
    ctx.qp_set_integrals(torch.from_numpy(s.h).to(dev), torch.from_numpy(s.eri).to(dev))
    E0 = torch.tensor([-1.0], dtype=torch.float64, device=dev)
    coefs = torch.from_numpy(s.coefs).to(dev)
    dup = s.dets.copy()
    dup[3] = dup[5]
    with pytest.raises(QPError) as e:
        ctx.pt2(to_device_dets(dup, dev), coefs, E0)
    assert e.value.code == _lib.QP_E_DUP
    bad = s.dets.copy()
    bad[2, 0, 0] |= np.uint64(1) << np.uint64(40)   # orbital 40 >= n_orb and one extra electron
    with pytest.raises(QPError) as e:
        ctx.pt2(to_device_dets(bad, dev), coefs, E0)
    assert e.value.code in (_lib.QP_E_NORB, _lib.QP_E_ELEC)
    elec = s.dets.copy()
    w = int(elec[4, 1, 0])
    p = max(q for q in range(s.n_orb) if not (w >> q) & 1)
    elec[4, 1, 0] = np.uint64(w | (1 << p))      # one extra down electron
    with pytest.raises(QPError) as e:
        ctx.pt2(to_device_dets(elec, dev), coefs, E0)
    assert e.value.code == _lib.QP_E_ELEC
    c5 = torch.zeros((5, s.n_det), dtype=torch.float64, device=dev)
    with pytest.raises(QPError) as e:
        ctx.pt2(to_device_dets(s.dets, dev), c5, torch.zeros(5, dtype=torch.float64, device=dev))
    assert e.value.code == _lib.QP_E_STATES
    fresh = Context(0)
    with pytest.raises(QPError) as e:
        fresh.pt2(to_device_dets(s.dets, dev), coefs, E0)
    assert e.value.code == _lib.QP_E_NOINT
    fresh.close()
    # empty wave function: E_PT2 = 0, nothing selected
    r = ctx.pt2(to_device_dets(s.dets[:0], dev), coefs[:, :0].contiguous(), E0, n_select=5)
    assert r["e_pt2"].item() == 0.0 and r["sel_dets"].shape[0] == 0
    # a generator list with an index outside [0, n_det) is refused
    with pytest.raises(QPError) as e:
        ctx.pt2_generators(to_device_dets(s.dets, dev), coefs, E0,
                           torch.tensor([0, s.n_det], dtype=torch.int32))
    assert e.value.code == _lib.QP_E_ARG
