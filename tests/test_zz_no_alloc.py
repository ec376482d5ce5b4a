"""qp_generator_order_noalloc (the entry point that allocates nothing: its
scratch is a file-scope device array) against qp_generator_order on the same
inputs: two calls in a row, the second smaller, bit-exact permutations; ties
of the weights sum_k c_k^2 broken by the determinant key alike; sizes beyond
its stated maximum rejected before any launch."""
import numpy as np
import pytest

from paper_1902_08154_amd import synth

pytestmark = pytest.mark.gpu


def _system(n, nu, nd, ndet, ns, seed, ties=False):
    s = synth.make_system(f"noalloc_n{n}", seed, n, nu, nd, ndet, n_states=ns)
    if ties:
        # coarse magnitudes: many determinants share sum_k c_k^2
        s.coefs = np.round(s.coefs, 2)
    return s


def test_noalloc_generator_order_matches_allocating_entry():
    import torch
    from paper_1902_08154_amd.api import Context, to_device_dets
    ctx = Context(0)
    dev = ctx.device
    # first a larger call, three words per spin and two states, then a smaller
    # one with one word and tied weights: the second must not see the first's
    # scratch contents
    for n, nu, nd, ndet, ns, seed, ties in [(130, 4, 4, 6000, 2, 901, False), (40, 5, 5, 2500, 1, 902, True)]:
        s = _system(n, nu, nd, ndet, ns, seed, ties)
        ctx.qp_set_integrals(torch.from_numpy(s.h).to(dev), torch.from_numpy(s.eri).to(dev))
        dets = to_device_dets(s.dets, dev)
        coefs = torch.from_numpy(np.ascontiguousarray(s.coefs)).to(dev)
        ref = torch.empty(s.n_det, dtype=torch.int32, device=dev)
        ctx.qp_generator_order(dets, coefs, ref)
        out = torch.full((s.n_det,), -7, dtype=torch.int32, device=dev)
        ctx.qp_generator_order_noalloc(dets, coefs, out)
        torch.cuda.synchronize()
        r, o = ref.cpu().numpy(), out.cpu().numpy()
        print(f"n={n} n_det={s.n_det} states={ns} ties={ties}: {int((r != o).sum())} positions differ")
        assert np.array_equal(r, o)
        assert np.array_equal(np.sort(o), np.arange(s.n_det))
    ctx.close()


def test_noalloc_generator_order_rejects_oversize():
    import torch
    from paper_1902_08154_amd import _lib
    from paper_1902_08154_amd.api import Context, QPError
    ctx = Context(0)
    dev = ctx.device
    s = _system(20, 3, 3, 50, 1, 903)
    ctx.qp_set_integrals(torch.from_numpy(s.h).to(dev), torch.from_numpy(s.eri).to(dev))
    n = _lib.QP_NOALLOC_MAX_DET + 1
    # sizes only: the entry point rejects them before reading any input
    dets = torch.zeros((n, 2, 1), dtype=torch.int64, device=dev)
    coefs = torch.zeros((1, n), dtype=torch.float64, device=dev)
    out = torch.empty(n, dtype=torch.int32, device=dev)
    with pytest.raises(QPError) as e:
        ctx.qp_generator_order_noalloc(dets, coefs, out)
    assert e.value.code == _lib.QP_E_ARG
    ctx.close()
