"""Python front end of the C ABI (same names, argument marshalling only)."""
import ctypes

import numpy as np

from . import _native as nat


def _stream_ptr(stream):
    """hipStream_t of a torch stream; None means torch's current stream (NULL,
    the legacy default stream, when no GPU is visible: argument errors are
    still reported before any device work)."""
    if stream is None:
        import torch
        if not torch.cuda.is_available():
            return ctypes.c_void_p(0)
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


class EriStore:
    """Owns one molecule's screened integral store in HBM (esmf_eri_prepare)."""

    def __init__(self, centers, exponents, tau, storage=nat.STORE_FP64, stream=None, lmn=None):
        """lmn: optional [N, 3] Cartesian powers (l, m, n) per function, l + m + n <= 2
        (esmf_eri_prepare_cart); None for s functions."""
        c = np.ascontiguousarray(centers, dtype=np.float64)
        a = np.ascontiguousarray(exponents, dtype=np.float64)
        if c.ndim != 2 or c.shape[1] != 3 or a.ndim != 1 or a.shape[0] != c.shape[0]:
            raise nat.InvalidArgument(nat.ESMF_ERR_INVALID_ARG, "ESMF_ERR_INVALID_ARG",
                                      "centers must be [N,3] and exponents [N]")
        self.nbf = int(a.shape[0])
        self.storage = int(storage)
        h = ctypes.c_void_p()
        L = nat.lib()
        if lmn is None:
            nat.check(L.esmf_eri_prepare(self.nbf, c.ctypes.data_as(nat._dp), a.ctypes.data_as(nat._dp),
                                         float(tau), self.storage, _stream_ptr(stream), ctypes.byref(h)))
        else:
            lm = np.ascontiguousarray(lmn, dtype=np.int32)
            if lm.shape != (self.nbf, 3):
                raise nat.InvalidArgument(nat.ESMF_ERR_INVALID_ARG, "ESMF_ERR_INVALID_ARG", "lmn must be [N,3]")
            nat.check(L.esmf_eri_prepare_cart(self.nbf, c.ctypes.data_as(nat._dp), a.ctypes.data_as(nat._dp),
                                              lm.ctypes.data_as(nat._i32p), float(tau), self.storage,
                                              _stream_ptr(stream), ctypes.byref(h)))
        self._h = h

    @classmethod
    def contracted(cls, centers, lmn, prim_offset, prim_exp, prim_coef, tau, storage=nat.STORE_FP64,
                   stream=None):
        """A store over contracted Cartesian functions (esmf_eri_prepare_contracted):
        function i is the normalised sum over primitives prim_offset[i] .. prim_offset[i+1]-1."""
        c = np.ascontiguousarray(centers, dtype=np.float64)
        lm = np.ascontiguousarray(lmn, dtype=np.int32)
        po = np.ascontiguousarray(prim_offset, dtype=np.int32)
        pe = np.ascontiguousarray(prim_exp, dtype=np.float64)
        pc = np.ascontiguousarray(prim_coef, dtype=np.float64)
        n = int(c.shape[0]) if c.ndim == 2 else -1
        if (c.ndim != 2 or c.shape[1] != 3 or lm.shape != (n, 3) or po.shape != (n + 1,)
                or pe.shape != (int(po[-1]),) or pc.shape != pe.shape):
            raise nat.InvalidArgument(nat.ESMF_ERR_INVALID_ARG, "ESMF_ERR_INVALID_ARG",
                                      "centers [N,3], lmn [N,3], prim_offset [N+1], prim_exp/coef [P]")
        self = cls.__new__(cls)
        self.nbf = n
        self.storage = int(storage)
        h = ctypes.c_void_p()
        nat.check(nat.lib().esmf_eri_prepare_contracted(
            n, c.ctypes.data_as(nat._dp), lm.ctypes.data_as(nat._i32p), po.ctypes.data_as(nat._i32p),
            pe.ctypes.data_as(nat._dp), pc.ctypes.data_as(nat._dp), float(tau), self.storage,
            _stream_ptr(stream), ctypes.byref(h)))
        self._h = h
        return self

    @property
    def handle(self):
        if self._h is None or not self._h.value:
            raise ValueError("EriStore released")
        return self._h

    def info(self):
        out = nat.EriInfo()
        nat.check(nat.lib().esmf_eri_info_get(self.handle, ctypes.byref(out)))
        return out.as_dict()

    def lookup(self, p, q, r, s):
        arrs = [np.ascontiguousarray(x, dtype=np.int32) for x in (p, q, r, s)]
        cnt = arrs[0].shape[0]
        out = np.empty(cnt)
        nat.check(nat.lib().esmf_eri_lookup(self.handle, cnt, *[x.ctypes.data_as(nat._i32p) for x in arrs],
                                            out.ctypes.data_as(nat._dp)))
        return out

    def release(self):
        if self._h is not None and self._h.value:
            nat.check(nat.lib().esmf_eri_release(self._h))
        self._h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


def _check_tensor(t, shape, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 \
            or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise nat.InvalidArgument(nat.ESMF_ERR_INVALID_ARG, "ESMF_ERR_INVALID_ARG",
                                  f"{name} must be a contiguous float64 CUDA tensor of shape {shape}")


# The paper's nine ESMF densities (nine_densities order): Theta^T Theta and A
# are symmetric.
ESMF_SYMMETRIC = (1, 0, 1, 0, 0, 0, 0, 0, 0)


def fock_build(store, d, j=None, k=None, prec=nat.PREC_FP64, stream=None, symmetric=None):
    """J[D_i], K[D_i] for d of shape [m, N, N] (esmf_fock_build).  Returns (j, k).
    symmetric: m flags marking exactly symmetric densities (esmf_fock_build_sym),
    which then take one matrix-core column instead of two."""
    import torch
    m = int(d.shape[0]) if d.dim() == 3 else -1
    n = store.nbf
    _check_tensor(d, (m, n, n), "d")
    if j is None:
        j = torch.empty_like(d)
    if k is None:
        k = torch.empty_like(d)
    _check_tensor(j, (m, n, n), "j")
    _check_tensor(k, (m, n, n), "k")
    if symmetric is None:
        nat.check(nat.lib().esmf_fock_build(store.handle, m, ctypes.c_void_p(d.data_ptr()),
                                            ctypes.c_void_p(j.data_ptr()), ctypes.c_void_p(k.data_ptr()),
                                            int(prec), _stream_ptr(stream)))
        return j, k
    flags = [int(bool(x)) for x in symmetric]
    if len(flags) != m:
        raise nat.InvalidArgument(nat.ESMF_ERR_INVALID_ARG, "ESMF_ERR_INVALID_ARG",
                                  f"symmetric must hold {m} flags")
    fl = (ctypes.c_uint8 * m)(*flags)
    nat.check(nat.lib().esmf_fock_build_sym(store.handle, m, ctypes.c_void_p(d.data_ptr()),
                                            ctypes.c_void_p(j.data_ptr()), ctypes.c_void_p(k.data_ptr()),
                                            int(prec), fl, _stream_ptr(stream)))
    return j, k


def fock_build_batched(stores, ds, js, ks, prec=nat.PREC_FP64, stream=None):
    """Many molecules in one launch (esmf_fock_build_batched)."""
    nmol = len(stores)
    for st, d, j, k in zip(stores, ds, js, ks):
        m = int(d.shape[0])
        for t, nm in ((d, "d"), (j, "j"), (k, "k")):
            _check_tensor(t, (m, st.nbf, st.nbf), nm)
    VP = ctypes.c_void_p * nmol
    hs = VP(*[st.handle.value for st in stores])
    ms = (ctypes.c_int32 * nmol)(*[int(d.shape[0]) for d in ds])
    dp = VP(*[d.data_ptr() for d in ds])
    jp = VP(*[j.data_ptr() for j in js])
    kp = VP(*[k.data_ptr() for k in ks])
    nat.check(nat.lib().esmf_fock_build_batched(nmol, hs, ms, dp, jp, kp, int(prec),
                                                _stream_ptr(stream)))
    return js, ks


def fock_tune(store, m, prec=nat.PREC_FP64, stream=None):
    """Time every contraction variant on this store and keep the fastest for
    its builds of that precision (esmf_fock_tune).  Returns the table."""
    rep = nat.TuneReport()
    nat.check(nat.lib().esmf_fock_tune(store.handle, int(m), int(prec), _stream_ptr(stream),
                                       ctypes.byref(rep)))
    return rep.as_dict()


def batched_report():
    """What this thread's last batched build ran (esmf_fock_batched_report):
    graph replay or not, units, items, the chosen variant and the tuner's
    table."""
    rep = nat.BatchReport()
    nat.check(nat.lib().esmf_fock_batched_report(ctypes.byref(rep)))
    return rep.as_dict()


def nine_densities(theta, gamma, sigma, mu, r, phi, d=None, stream=None):
    """The nine densities of one ESMF gradient evaluation (esmf_nine_densities)
    as a [9, N, N] float64 CUDA tensor.  theta [No, N], gamma [Nv, N],
    sigma and mu [No, Nv], r [No, N], phi [Nv, N]: contiguous float64 CUDA."""
    import torch
    no, n = (int(x) for x in theta.shape) if theta.dim() == 2 else (-1, -1)
    nv = int(gamma.shape[0]) if gamma.dim() == 2 else -1
    for t, shape, name in ((theta, (no, n), "theta"), (gamma, (nv, n), "gamma"), (sigma, (no, nv), "sigma"),
                           (mu, (no, nv), "mu"), (r, (no, n), "r"), (phi, (nv, n), "phi")):
        _check_tensor(t, shape, name)
    if d is None:
        d = torch.empty((9, n, n), dtype=torch.float64, device=theta.device)
    _check_tensor(d, (9, n, n), "d")
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    nat.check(nat.lib().esmf_nine_densities(n, no, nv, ptr(theta), ptr(gamma), ptr(sigma), ptr(mu), ptr(r),
                                            ptr(phi), ptr(d), _stream_ptr(stream)))
    return d


def energy_two_body(d, j, k, n2, c0, stream=None):
    """E_2 of Eq. esmf_energy_2b (esmf_energy_two_body),
    N2 F[D1].D1 + 4 c0 F[D1].D2 + 2 F[D1].A + 2 F[D2].D2, from D1, D2, A (the
    first three of d) and the J, K of D1 and D2: a 0-dim float64 CUDA tensor,
    written asynchronously on the stream."""
    import torch
    n = int(d.shape[-1])
    for t, name, lo in ((d, "d", 3), (j, "j", 2), (k, "k", 2)):
        if t.dim() != 3 or t.shape[0] < lo:
            raise nat.InvalidArgument(nat.ESMF_ERR_INVALID_ARG, "ESMF_ERR_INVALID_ARG",
                                      f"{name} must hold at least {lo} [N, N] matrices")
        _check_tensor(t, (int(t.shape[0]), n, n), name)
    e2 = torch.empty((), dtype=torch.float64, device=d.device)
    nat.check(nat.lib().esmf_energy_two_body(n, float(n2), float(c0), ctypes.c_void_p(d.data_ptr()),
                                             ctypes.c_void_p(j.data_ptr()), ctypes.c_void_p(k.data_ptr()),
                                             ctypes.c_void_p(e2.data_ptr()), _stream_ptr(stream)))
    return e2


def energy_gradient(theta, gamma, sigma, g, d, j, k, c0, n2, stream=None):
    """The ESMF energy and its first derivatives (esmf_energy_gradient) from
    the J, K of D1, D2, A.  Returns dict(energy=[E_1, E_2, E, dE/dc0] as a
    float64 CUDA tensor, sigma, theta, gamma: the derivative tensors)."""
    import torch
    no, n = (int(x) for x in theta.shape) if theta.dim() == 2 else (-1, -1)
    nv = int(gamma.shape[0]) if gamma.dim() == 2 else -1
    for t, shape, name in ((theta, (no, n), "theta"), (gamma, (nv, n), "gamma"), (sigma, (no, nv), "sigma"),
                           (g, (n, n), "g")):
        _check_tensor(t, shape, name)
    for t, name in ((d, "d"), (j, "j"), (k, "k")):
        if t.dim() != 3 or t.shape[0] < 3:
            raise nat.InvalidArgument(nat.ESMF_ERR_INVALID_ARG, "ESMF_ERR_INVALID_ARG",
                                      f"{name} must hold at least 3 [N, N] matrices")
        _check_tensor(t, (int(t.shape[0]), n, n), name)
    out = dict(energy=torch.empty(4, dtype=torch.float64, device=theta.device),
               sigma=torch.empty_like(sigma), theta=torch.empty_like(theta), gamma=torch.empty_like(gamma))
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    nat.check(nat.lib().esmf_energy_gradient(n, no, nv, float(c0), float(n2), ptr(theta), ptr(gamma), ptr(sigma),
                                             ptr(g), ptr(d), ptr(j), ptr(k), ptr(out["energy"]),
                                             ptr(out["sigma"]), ptr(out["theta"]), ptr(out["gamma"]),
                                             _stream_ptr(stream)))
    return out


class Server:
    """Serving loop (esmf_server_*): sessions admitted against an HBM budget,
    continuous grouping of build requests over several streams."""

    def __init__(self, prec=nat.PREC_FP64, nstreams=4, max_group=16, max_inflight=2,
                 hbm_budget_bytes=200 * 10**9, workspace_limit_bytes=16 * 10**9, storage=None):
        if storage is None:
            storage = nat.STORE_FP64 if prec == nat.PREC_FP64 else nat.STORE_FP32
        cfg = nat.ServerConfig(nstreams=nstreams, max_group=max_group, max_inflight=max_inflight,
                               prec=int(prec), storage=int(storage),
                               reserved=0, hbm_budget_bytes=int(hbm_budget_bytes),
                               workspace_limit_bytes=int(workspace_limit_bytes))
        h = ctypes.c_void_p()
        nat.check(nat.lib().esmf_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self.prec = prec

    @property
    def handle(self):
        if self._h is None or not self._h.value:
            raise ValueError("Server destroyed")
        return self._h

    def open_session(self, centers, exponents, tau):
        """Returns (session id, footprint bytes); raises OutOfMemory (with
        .footprint set) when the store does not fit in the budget left."""
        c = np.ascontiguousarray(centers, dtype=np.float64)
        a = np.ascontiguousarray(exponents, dtype=np.float64)
        if c.ndim != 2 or c.shape[1] != 3 or a.ndim != 1 or a.shape[0] != c.shape[0]:
            raise nat.InvalidArgument(nat.ESMF_ERR_INVALID_ARG, "ESMF_ERR_INVALID_ARG",
                                      "centers must be [N,3] and exponents [N]")
        sid = ctypes.c_int32()
        fp = ctypes.c_int64()
        st = nat.lib().esmf_server_open_session(self.handle, int(a.shape[0]), c.ctypes.data_as(nat._dp),
                                                a.ctypes.data_as(nat._dp), float(tau),
                                                ctypes.byref(sid), ctypes.byref(fp))
        try:
            nat.check(st)
        except nat.EsmfError as e:
            e.footprint = fp.value
            raise
        return sid.value, fp.value

    def open_session_contracted(self, centers, lmn, prim_offset, prim_exp, prim_coef, tau):
        """A session over contracted Cartesian functions
        (esmf_server_open_session_contracted); returns as open_session."""
        c = np.ascontiguousarray(centers, dtype=np.float64)
        lm = np.ascontiguousarray(lmn, dtype=np.int32)
        po = np.ascontiguousarray(prim_offset, dtype=np.int32)
        pe = np.ascontiguousarray(prim_exp, dtype=np.float64)
        pc = np.ascontiguousarray(prim_coef, dtype=np.float64)
        n = int(c.shape[0]) if c.ndim == 2 else -1
        if (c.ndim != 2 or c.shape[1] != 3 or lm.shape != (n, 3) or po.shape != (n + 1,)
                or pe.shape != (int(po[-1]),) or pc.shape != pe.shape):
            raise nat.InvalidArgument(nat.ESMF_ERR_INVALID_ARG, "ESMF_ERR_INVALID_ARG",
                                      "centers [N,3], lmn [N,3], prim_offset [N+1], prim_exp/coef [P]")
        sid = ctypes.c_int32()
        fp = ctypes.c_int64()
        st = nat.lib().esmf_server_open_session_contracted(
            self.handle, n, c.ctypes.data_as(nat._dp), lm.ctypes.data_as(nat._i32p), po.ctypes.data_as(nat._i32p),
            pe.ctypes.data_as(nat._dp), pc.ctypes.data_as(nat._dp), float(tau), ctypes.byref(sid), ctypes.byref(fp))
        try:
            nat.check(st)
        except nat.EsmfError as e:
            e.footprint = fp.value
            raise
        return sid.value, fp.value

    def close_session(self, session):
        nat.check(nat.lib().esmf_server_close_session(self.handle, int(session)))

    def submit(self, session, d, j, k, stream=None):
        """Queue a build of d [m, N, N] into j, k (device tensors kept alive by
        the caller until wait); returns the request id.  The build follows
        the work enqueued on `stream` (default: torch's current stream)
        before this call, e.g. the kernels that wrote d."""
        m = int(d.shape[0])
        n = int(d.shape[1])
        for t, nm in ((d, "d"), (j, "j"), (k, "k")):
            _check_tensor(t, (m, n, n), nm)
        rid = ctypes.c_int64()
        nat.check(nat.lib().esmf_server_submit(self.handle, int(session), m, ctypes.c_void_p(d.data_ptr()),
                                               ctypes.c_void_p(j.data_ptr()), ctypes.c_void_p(k.data_ptr()),
                                               _stream_ptr(stream), ctypes.byref(rid)))
        return rid.value

    def wait(self, request):
        """Block until the request completed; returns its latency in ms."""
        lat = ctypes.c_double()
        nat.check(nat.lib().esmf_server_wait(self.handle, int(request), ctypes.byref(lat)))
        return lat.value

    def stats(self):
        out = nat.ServerStats()
        nat.check(nat.lib().esmf_server_stats_get(self.handle, ctypes.byref(out)))
        return out.as_dict()

    def destroy(self):
        if self._h is not None and self._h.value:
            nat.check(nat.lib().esmf_server_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def timing_enable(on=True):
    """Record HIP events around each build's main contraction kernel."""
    nat.check(nat.lib().esmf_timing_enable(1 if on else 0))


def timing_collect():
    """(summed ms, number of timed builds) since the previous collect."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    nat.check(nat.lib().esmf_timing_collect(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def probe_peaks(copy_bytes=2 << 30, stream=None):
    """Measured FP64 matrix-core and vector FMA rates (TFLOP/s) and the rate
    of a streaming device copy (TB/s, read + written) of the current device."""
    out = nat.Peaks()
    nat.check(nat.lib().esmf_probe_peaks(int(copy_bytes), _stream_ptr(stream), ctypes.byref(out)))
    return out.as_dict()
