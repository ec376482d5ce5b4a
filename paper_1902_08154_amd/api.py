"""Thin Python binding over the C ABI: argument marshalling only.

Every function takes torch tensors that already live on the context's HIP
device and passes their raw pointers and the current stream to libqp_pt2.so.
Determinant bit strings are carried in torch.int64 tensors (same bits as the
uint64 words of the ABI) of shape [n_det, 2, n_int].
"""
from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import _lib


class QPError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_lib.ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _need(t: torch.Tensor, dtype, name: str, device):
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor on the GPU")
    if t.device != device:
        raise TypeError(f"{name} is on {t.device}, context is on {device}")


class Context:
    """Owns one qp_ctx (device layouts of the integrals and scratch)."""

    def __init__(self, device: int = 0):
        self._lib = _lib.load()
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        rc = self._lib.qp_create(ctypes.byref(h), device)
        if rc != 0:
            raise QPError(rc, "qp_create failed")
        self._h = h
        self.n_orb = 0

    def close(self):
        if getattr(self, "_h", None):
            self._lib.qp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int):
        if rc != 0:
            msg = self._lib.qp_last_error(self._h).decode()
            raise QPError(rc, msg)

    # ------------------------------------------------------------------ ABI
    def qp_set_integrals(self, h: torch.Tensor, eri_packed: torch.Tensor):
        _need(h, torch.float64, "h", self.device)
        _need(eri_packed, torch.float64, "eri_packed", self.device)
        n = h.shape[0]
        self._check(self._lib.qp_set_integrals(self._h, _ptr(h), _ptr(eri_packed), n, _stream(self.device)))
        self.n_orb = n
        self._ints_src = None

    def ensure_integrals(self, h: torch.Tensor, eri_packed: torch.Tensor):
        """qp_set_integrals unless the last tensors set through this method
        occupy the same memory (address, shape) and have not been modified in
        place since (same version counter).  The context keeps references to
        those tensors, so their memory cannot be freed and handed to another
        tensor at the same address meanwhile: a match is the same storage."""
        key = (h.data_ptr(), h._version, tuple(h.shape), eri_packed.data_ptr(), eri_packed._version,
               eri_packed.numel())
        src = getattr(self, "_ints_src", None)
        if src is not None and src[2] == key:
            return
        self.qp_set_integrals(h.detach(), eri_packed.detach())
        self._ints_src = (h.detach(), eri_packed.detach(), key)

    def qp_pt2(self, dets, coefs, E0, n_select=0, flags=0, e_pt2=None, sel_dets=None, sel_e=None,
               n_sel=None, stats=None, eps_gen=None):
        self._check(self._lib.qp_pt2(self._h, _ptr(dets), _ptr(coefs), dets.shape[0], coefs.shape[0],
                                     _ptr(E0), n_select, flags, _ptr(e_pt2), _ptr(sel_dets), _ptr(sel_e),
                                     _ptr(n_sel), _ptr(stats), _ptr(eps_gen), _stream(self.device)))

    def qp_pt2_backward(self, dets, coefs, E0, grad_e_pt2, flags=0, grad_coefs=None, grad_E0=None,
                        grad_h=None, stats=None):
        self._check(self._lib.qp_pt2_backward(self._h, _ptr(dets), _ptr(coefs), dets.shape[0],
                                              coefs.shape[0], _ptr(E0), _ptr(grad_e_pt2), flags,
                                              _ptr(grad_coefs), _ptr(grad_E0), _ptr(grad_h), _ptr(stats),
                                              _stream(self.device)))

    def qp_generator_order(self, dets, coefs, order_out, flags=0):
        self._check(self._lib.qp_generator_order(self._h, _ptr(dets), _ptr(coefs), dets.shape[0], coefs.shape[0],
                                                 flags, _ptr(order_out), _stream(self.device)))

    def qp_generator_order_noalloc(self, dets, coefs, order_out, flags=0):
        self._check(self._lib.qp_generator_order_noalloc(self._h, _ptr(dets), _ptr(coefs), dets.shape[0],
                                                         coefs.shape[0], flags, _ptr(order_out),
                                                         _stream(self.device)))

    def qp_pt2_generators(self, dets, coefs, E0, gens, n_select=0, flags=0, eps_out=None, sel_dets=None,
                          sel_e=None, n_sel=None, stats=None):
        self._check(self._lib.qp_pt2_generators(self._h, _ptr(dets), _ptr(coefs), dets.shape[0], coefs.shape[0],
                                                _ptr(E0), _ptr(gens), gens.numel(), n_select, flags,
                                                _ptr(eps_out), _ptr(sel_dets), _ptr(sel_e), _ptr(n_sel),
                                                _ptr(stats), _stream(self.device)))

    def qp_pt2_stochastic(self, dets, coefs, E0, uniforms, rel_err, det_chunk, draws_per_round, flags=0,
                          n_select=0, sel_dets=None, sel_e=None, n_sel=None, computed=None):
        """uniforms: host float64 numpy array.  Returns (e_est, e_err, n_computed, n_rounds);
        with n_select > 0 the selection goes to the device tensors sel_dets, sel_e, n_sel."""
        import numpy as np
        ns = coefs.shape[0]
        u = np.ascontiguousarray(uniforms, dtype=np.float64)
        e = np.zeros(ns)
        err = np.zeros(ns)
        nc = np.zeros(1, dtype=np.int64)
        nr = np.zeros(1, dtype=np.int64)
        hp = lambda a: ctypes.c_void_p(a.ctypes.data)
        self._check(self._lib.qp_pt2_stochastic(self._h, _ptr(dets), _ptr(coefs), dets.shape[0], ns, _ptr(E0),
                                                hp(u) if u.size else None, u.size, float(rel_err), int(det_chunk),
                                                int(draws_per_round), int(n_select), flags, hp(e), hp(err), hp(nc),
                                                hp(nr), _ptr(sel_dets), _ptr(sel_e), _ptr(n_sel), _ptr(computed),
                                                _stream(self.device)))
        return e, err, int(nc[0]), int(nr[0])

    def qp_sigma(self, dets, U, W, flags=0):
        self._check(self._lib.qp_sigma(self._h, _ptr(dets), dets.shape[0], U.shape[0], _ptr(U), flags, _ptr(W),
                                       _stream(self.device)))

    def qp_davidson(self, dets, n_states, guess, tol, max_iter, C_out, flags=0):
        """Returns (E [ns] numpy, <S^2> [ns] numpy, iterations); C_out is filled."""
        import numpy as np
        e = np.zeros(n_states)
        s2 = np.zeros(n_states)
        it = (ctypes.c_int * 1)()
        hp = lambda a: ctypes.c_void_p(a.ctypes.data)
        self._check(self._lib.qp_davidson(self._h, _ptr(dets), dets.shape[0], n_states, _ptr(guess), float(tol),
                                          int(max_iter), flags, hp(e), _ptr(C_out), hp(s2), it,
                                          _stream(self.device)))
        return e, s2, int(it[0])

    def qp_pt2_batched(self, systems, with_backward=False, flags=0):
        """systems: a sequence of _lib.System records."""
        arr = (_lib.System * max(len(systems), 1))(*systems)
        self._check(self._lib.qp_pt2_batched(self._h, len(systems), arr, 1 if with_backward else 0, flags,
                                             _stream(self.device)))

    def qp_energy(self, dets, coefs, E0_out, flags=0):
        self._check(self._lib.qp_energy(self._h, _ptr(dets), _ptr(coefs), dets.shape[0], coefs.shape[0],
                                        flags, _ptr(E0_out), _stream(self.device)))

    def qp_set_timing(self, enable: bool):
        self._check(self._lib.qp_set_timing(self._h, 1 if enable else 0))

    def qp_last_timing(self):
        """(dense sweep kernel ms, general kernel ms, whole call ms, clean-cell and
        split-correction kernels ms, clean-cell kernel ms) of the last timed call."""
        out = (ctypes.c_double * 5)()
        self._check(self._lib.qp_last_timing(self._h, out))
        return tuple(float(out[i]) for i in range(5))

    def qp_alu_probe(self, kind, iters=1 << 14):
        """Vector-ALU lane operations per second this device issues for
        `kind` (_lib.QP_PROBE_F64_FMA / I32_ADD / MIXED), on the current
        stream."""
        out = ctypes.c_double(0.0)
        self._check(self._lib.qp_alu_probe(self._h, int(kind), int(iters), _stream(self.device),
                                           ctypes.byref(out)))
        return float(out.value)

    def qp_set_split(self, mode):
        """mode: _lib.QP_SPLIT_NEVER / AUTO / ALWAYS; True and False stand for
        ALWAYS and NEVER."""
        if mode is True:
            mode = _lib.QP_SPLIT_ALWAYS
        elif mode is False:
            mode = _lib.QP_SPLIT_NEVER
        self._check(self._lib.qp_set_split(self._h, int(mode)))

    # ---------------------------------------------------------- conveniences
    def _inputs(self, dets, coefs, E0=None):
        _need(dets, torch.int64, "dets", self.device)
        if dets.dim() != 3 or dets.shape[1] != 2:
            raise ValueError("dets must have shape [n_det, 2, n_int]")
        _need(coefs, torch.float64, "coefs", self.device)
        if coefs.dim() != 2 or coefs.shape[1] != dets.shape[0]:
            raise ValueError("coefs must have shape [n_states, n_det]")
        if E0 is not None:
            _need(E0, torch.float64, "E0", self.device)
            if E0.numel() != coefs.shape[0]:
                raise ValueError("E0 must have n_states entries")

    def pt2(self, dets, coefs, E0, n_select=0, eps_gen=False, fingerprint=False, check=True):
        """Forward sweep.  Returns a dict with e_pt2 [ns], sel_dets [m,2,nint],
        sel_e [m,ns], stats (dict) and optionally eps_gen [ns, n_det]."""
        self._inputs(dets, coefs, E0)
        ns, nd = coefs.shape
        dev = self.device
        e = torch.empty(ns, dtype=torch.float64, device=dev)
        st = torch.zeros(ctypes.sizeof(_lib.Stats), dtype=torch.uint8, device=dev)
        sd = torch.empty((max(n_select, 1), 2, dets.shape[2]), dtype=torch.int64, device=dev)
        se = torch.empty((max(n_select, 1), ns), dtype=torch.float64, device=dev)
        nsel = torch.zeros(1, dtype=torch.int64, device=dev)
        eg = torch.empty((ns, nd), dtype=torch.float64, device=dev) if eps_gen else None
        flags = (_lib.QP_FLAG_FINGERPRINT if fingerprint else 0) | (0 if check else _lib.QP_FLAG_NOCHECK)
        self.qp_pt2(dets, coefs, E0, n_select, flags, e, sd if n_select > 0 else None,
                    se if n_select > 0 else None, nsel if n_select > 0 else None, st, eg)
        m = int(nsel.item()) if n_select > 0 else 0
        out = dict(e_pt2=e, sel_dets=sd[:m], sel_e=se[:m], stats=stats_to_dict(st, ns))
        if eps_gen:
            out["eps_gen"] = eg
        return out

    def pt2_backward(self, dets, coefs, E0, grad_e_pt2, want=("coefs", "E0", "h")):
        self._inputs(dets, coefs, E0)
        ns, nd = coefs.shape
        dev = self.device
        gc = torch.empty((ns, nd), dtype=torch.float64, device=dev) if "coefs" in want else None
        gE = torch.empty(ns, dtype=torch.float64, device=dev) if "E0" in want else None
        gh = torch.empty((self.n_orb, self.n_orb), dtype=torch.float64, device=dev) if "h" in want else None
        g = grad_e_pt2.to(device=dev, dtype=torch.float64).contiguous()
        self.qp_pt2_backward(dets, coefs, E0, g, 0, gc, gE, gh, None)
        return gc, gE, gh

    def generator_order(self, dets, coefs):
        """Determinant indices in generator order (torch.int32 on the device)."""
        self._inputs(dets, coefs)
        out = torch.empty(dets.shape[0], dtype=torch.int32, device=self.device)
        self.qp_generator_order(dets, coefs, out)
        return out

    def pt2_generators(self, dets, coefs, E0, gens, n_select=0, fingerprint=False):
        """eps_I [ns, len(gens)] of the listed generators (determinant indices),
        with stats and, when n_select > 0, their selected alpha."""
        self._inputs(dets, coefs, E0)
        gens = gens.to(device=self.device, dtype=torch.int32).contiguous()
        ns = coefs.shape[0]
        dev = self.device
        eps = torch.empty((ns, max(gens.numel(), 1)), dtype=torch.float64, device=dev)
        st = torch.zeros(ctypes.sizeof(_lib.Stats), dtype=torch.uint8, device=dev)
        sd = torch.empty((max(n_select, 1), 2, dets.shape[2]), dtype=torch.int64, device=dev)
        se = torch.empty((max(n_select, 1), ns), dtype=torch.float64, device=dev)
        nsel = torch.zeros(1, dtype=torch.int64, device=dev)
        flags = _lib.QP_FLAG_FINGERPRINT if fingerprint else 0
        self.qp_pt2_generators(dets, coefs, E0, gens, n_select, flags, eps, sd if n_select > 0 else None,
                               se if n_select > 0 else None, nsel if n_select > 0 else None, st)
        m = int(nsel.item()) if n_select > 0 else 0
        return dict(eps=eps[:, :gens.numel()], stats=stats_to_dict(st, ns), sel_dets=sd[:m], sel_e=se[:m])

    def pt2_stochastic(self, dets, coefs, E0, uniforms, rel_err=0.002, det_chunk=None, draws_per_round=None,
                       n_select=0):
        """Semi-stochastic E_PT2.  uniforms: host random numbers in [0, 1), one
        per draw.  Returns dict(e_pt2, err, n_computed, n_rounds, computed);
        with n_select > 0 also the selection over the computed generators,
        made during the same sweeps: sel_dets, sel_e (trimmed to its length)."""
        self._inputs(dets, coefs, E0)
        n = dets.shape[0]
        # rounds large enough to keep the device busy: each one is a sweep launch
        # followed by a host decision
        if det_chunk is None:
            det_chunk = max(1, n // 40)
        if draws_per_round is None:
            draws_per_round = max(16, 4 * det_chunk)
        dev = self.device
        computed = torch.zeros(n, dtype=torch.uint8, device=dev)
        sd = se = nsl = None
        if n_select > 0:
            sd = torch.zeros((n_select,) + tuple(dets.shape[1:]), dtype=dets.dtype, device=dev)
            se = torch.zeros((n_select, coefs.shape[0]), dtype=torch.float64, device=dev)
            nsl = torch.zeros(1, dtype=torch.int64, device=dev)
        e, err, nc, nr = self.qp_pt2_stochastic(dets, coefs, E0, uniforms, rel_err, det_chunk, draws_per_round,
                                                n_select=n_select, sel_dets=sd, sel_e=se, n_sel=nsl,
                                                computed=computed)
        out = dict(e_pt2=e, err=err, n_computed=nc, n_rounds=nr, computed=computed.bool())
        if n_select > 0:
            m = int(nsl.item())
            out["sel_dets"], out["sel_e"] = sd[:m], se[:m]
        return out

    def sigma(self, dets, U, s2=False, reuse=False):
        """W = H U (or S^2 U) for U [n_vec, n_det] on the device.  reuse: the
        caller vouches that `dets` is unchanged since the previous sigma call
        with the same tensor (QP_SIGMA_REUSE)."""
        _need(dets, torch.int64, "dets", self.device)
        U = U.to(device=self.device, dtype=torch.float64).contiguous()
        W = torch.empty_like(U)
        self.qp_sigma(dets, U, W, (_lib.QP_SIGMA_S2 if s2 else 0) | (_lib.QP_SIGMA_REUSE if reuse else 0))
        return W

    def davidson(self, dets, n_states=1, guess=None, tol=1e-9, max_iter=200):
        """Lowest eigenpairs of H in the determinant space: dict(E, C [ns, n_det], s2, n_iter)."""
        _need(dets, torch.int64, "dets", self.device)
        C = torch.empty((n_states, dets.shape[0]), dtype=torch.float64, device=self.device)
        if guess is not None:
            guess = guess.to(device=self.device, dtype=torch.float64).contiguous()
        e, s2, it = self.qp_davidson(dets, n_states, guess, tol, max_iter, C)
        return dict(E=e, C=C, s2=s2, n_iter=it)

    def pt2_batched(self, systems, with_backward=False, fingerprint=False, check=True, reuse_integrals=False):
        """Many systems in one call.  `systems` is a sequence of dicts with
        tensors h [n,n], eri_packed, dets [n_det,2,n_int], coefs [ns,n_det],
        E0 [ns], and optionally n_select (forward only), eps_gen (bool) and,
        with_backward, grad_e_pt2 [ns] (default ones).  Returns one dict per
        system: e_pt2, stats, sel_dets/sel_e when n_select > 0, eps_gen if
        asked, and grad_coefs/grad_E0/grad_h with_backward."""
        dev = self.device
        recs, outs = [], []
        for i, y in enumerate(systems):
            h, eri, dets, coefs, E0 = y["h"], y["eri_packed"], y["dets"], y["coefs"], y["E0"]
            _need(h, torch.float64, f"systems[{i}].h", dev)
            _need(eri, torch.float64, f"systems[{i}].eri_packed", dev)
            self._inputs(dets, coefs, E0)
            n = h.shape[0]
            ns, nd = coefs.shape
            k = int(y.get("n_select", 0) or 0)
            o = dict(e_pt2=torch.empty(ns, dtype=torch.float64, device=dev),
                     stats=torch.zeros(ctypes.sizeof(_lib.Stats), dtype=torch.uint8, device=dev))
            r = _lib.System(n_orb=n, n_states=ns, n_det=nd, h=h.data_ptr(), eri_packed=eri.data_ptr(),
                            dets=dets.data_ptr(), coefs=coefs.data_ptr(), E0=E0.data_ptr(), n_select=k,
                            e_pt2=o["e_pt2"].data_ptr(), stats=o["stats"].data_ptr())
            if k > 0:
                o["sel_dets"] = torch.empty((k, 2, dets.shape[2]), dtype=torch.int64, device=dev)
                o["sel_e"] = torch.empty((k, ns), dtype=torch.float64, device=dev)
                o["n_sel"] = torch.zeros(1, dtype=torch.int64, device=dev)
                r.sel_dets, r.sel_e, r.n_sel = (o["sel_dets"].data_ptr(), o["sel_e"].data_ptr(),
                                                o["n_sel"].data_ptr())
            if y.get("eps_gen") and not with_backward:
                o["eps_gen"] = torch.empty((ns, nd), dtype=torch.float64, device=dev)
                r.eps_gen = o["eps_gen"].data_ptr()
            if with_backward:
                g = y.get("grad_e_pt2")
                g = torch.ones(ns, dtype=torch.float64, device=dev) if g is None else \
                    g.to(device=dev, dtype=torch.float64).contiguous()
                o["_g"] = g
                o["grad_coefs"] = torch.empty((ns, nd), dtype=torch.float64, device=dev)
                o["grad_E0"] = torch.empty(ns, dtype=torch.float64, device=dev)
                o["grad_h"] = torch.empty((n, n), dtype=torch.float64, device=dev)
                r.grad_e_pt2 = g.data_ptr()
                r.grad_coefs, r.grad_E0, r.grad_h = (o["grad_coefs"].data_ptr(), o["grad_E0"].data_ptr(),
                                                     o["grad_h"].data_ptr())
            recs.append(r)
            outs.append((o, ns, k))
        flags = ((_lib.QP_FLAG_FINGERPRINT if fingerprint else 0) | (0 if check else _lib.QP_FLAG_NOCHECK) |
                 (_lib.QP_FLAG_REUSE_INTEGRALS if reuse_integrals else 0))
        self.qp_pt2_batched(recs, with_backward, flags)
        res = []
        for o, ns, k in outs:
            o.pop("_g", None)
            o["stats"] = stats_to_dict(o["stats"], ns)
            if k > 0:
                m = int(o.pop("n_sel").item())
                o["sel_dets"], o["sel_e"] = o["sel_dets"][:m], o["sel_e"][:m]
            res.append(o)
        return res

    def energy(self, dets, coefs):
        self._inputs(dets, coefs)
        out = torch.empty(coefs.shape[0], dtype=torch.float64, device=self.device)
        self.qp_energy(dets, coefs, out)
        return out


class PT2Function(torch.autograd.Function):
    """E_PT2 per state (eqs. e2, PT2) as a differentiable function of the
    coefficients, E0 and the one-electron integrals h.

    forward runs qp_pt2; backward runs qp_pt2_backward with the upstream
    gradient, whose kernels recompute every numerator instead of storing them.
    Gradients are the library's partial derivatives (E0 independent, the alpha
    set fixed); dE/dh is the symmetric matrix G with dE = sum G_pq dh_pq for a
    symmetric dh.  The context's integrals are (re)built from (h, eri_packed)
    when either tensor changed since the last call.  Use through pt2_autograd().
    """

    @staticmethod
    def forward(fctx, context, dets, coefs, E0, h, eri_packed):
        context.ensure_integrals(h, eri_packed)
        e = context.pt2(dets, coefs, E0)["e_pt2"]
        fctx.context = context
        # the integrals travel with the graph node: another forward, or a
        # qp_set_integrals, between this forward and its backward must not
        # change the Hamiltonian the backward differentiates
        fctx.save_for_backward(dets, coefs, E0, h, eri_packed)
        return e

    @staticmethod
    def backward(fctx, grad_e):
        dets, coefs, E0, h, eri_packed = fctx.saved_tensors
        fctx.context.ensure_integrals(h, eri_packed)
        want = tuple(name for name, need in zip(("coefs", "E0", "h"), fctx.needs_input_grad[2:5]) if need)
        gc, gE, gh = fctx.context.pt2_backward(dets, coefs, E0, grad_e, want=want)
        return None, None, gc, gE, gh, None


def pt2_autograd(context, dets, coefs, E0, h, eri_packed):
    """E_PT2 [n_states], differentiable in coefs, E0 and h (see PT2Function)."""
    return PT2Function.apply(context, dets, coefs, E0, h, eri_packed)


def stats_to_dict(st: torch.Tensor, ns: int) -> dict:
    raw = bytes(st.cpu().numpy().tobytes())
    s = _lib.Stats.from_buffer_copy(raw)
    return dict(n_alpha=int(s.n_alpha), n_cells=int(s.n_cells), fingerprint=int(s.fingerprint),
                n_coarse=int(s.n_coarse), n_candidates=int(s.n_candidates), overflow=int(s.overflow),
                n_connections=int(s.n_connections), n_alpha_general=int(s.n_alpha_general),
                S=[float(s.S[k]) for k in range(ns)],
                min_abs_delta=float(s.min_abs_delta),
                Z=[float(s.Z[k]) for k in range(ns)], e_rpt2=[float(s.e_rpt2[k]) for k in range(ns)],
                n_fine=int(s.n_fine), n_alpha_clean=int(s.n_alpha_clean))


def to_device_dets(dets_u64, device) -> torch.Tensor:
    """numpy uint64 [n_det,2,n_int] -> torch.int64 on device (same bits)."""
    import numpy as np
    a = np.ascontiguousarray(dets_u64, dtype=np.uint64).view(np.int64)
    return torch.from_numpy(a.copy()).to(device)


def from_device_dets(t: torch.Tensor):
    import numpy as np
    return t.cpu().numpy().view(np.uint64)
