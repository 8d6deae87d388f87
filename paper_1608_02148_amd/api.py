"""Torch-facing wrappers of the C ABI (device memory and streams only).

Every step of the computation runs in the HIP library; these functions only
check shapes, allocate outputs / workspace as torch tensors and pass raw device
pointers together with torch's current HIP stream.
"""
import ctypes

import torch

from . import lib as L

_DTYPES = {torch.float64: L.RSVD_F64, torch.float32: L.RSVD_F32, torch.bfloat16: L.RSVD_BF16}

_handles = {}


def handle(device=None):
    """Per-device library handle bound to torch's current stream."""
    lib = L.load()
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    h = _handles.get(idx)
    if h is None:
        h = ctypes.c_void_p()
        with torch.cuda.device(idx):
            L.check(lib.rsvd_create(ctypes.byref(h), None), "rsvd_create")
        _handles[idx] = h
        _apply_tuned_variants(lib, h, idx)
    with torch.cuda.device(idx):
        stream = torch.cuda.current_stream(idx).cuda_stream
    L.check(lib.rsvd_set_stream(h, ctypes.c_void_p(stream)), "rsvd_set_stream")
    return h


def _apply_tuned_variants(lib, h, idx):
    """Apply the autotuned tile variants for this GPU's architecture, if the
    cache (paper_1608_02148_amd/tile_variants.json or $RSVD_TILE_VARIANTS)
    has an entry for it; otherwise the library's defaults stay."""
    import json
    import os
    path = os.environ.get("RSVD_TILE_VARIANTS",
                          os.path.join(os.path.dirname(os.path.abspath(__file__)), "tile_variants.json"))
    try:
        arch = torch.cuda.get_device_properties(idx).gcnArchName.split(":")[0]
        table = json.load(open(path))[arch]["f32"]
        if len(table) == 12:
            v = (ctypes.c_int32 * 12)(*[int(x) for x in table])
            lib.rsvd_set_tile_variants(h, v)
    except (OSError, KeyError, ValueError, TypeError):
        pass


def make_params(p=10, q=2, seed=0, stream_id=0, sdist="normal", precision="plain", probes=0, scheme="qr"):
    prm = L.Params()
    L.load().rsvd_default_params(ctypes.byref(prm))
    prm.p, prm.q, prm.seed, prm.stream_id = int(p), int(q), int(seed), int(stream_id)
    prm.probes = int(probes)
    prm.sdist = L.SDIST[sdist]
    prm.precision = L.PRECISION[precision]
    prm.scheme = L.SCHEME[scheme]
    return prm


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _check_matrix(A):
    if not isinstance(A, torch.Tensor) or A.dim() != 2 or not A.is_cuda:
        raise ValueError("A must be a 2-D tensor on a GPU")
    if A.dtype not in _DTYPES:
        raise ValueError(f"unsupported dtype {A.dtype}")
    if A.stride(1) != 1:
        raise ValueError("A must be row-major (unit stride along columns)")
    return _DTYPES[A.dtype]


def out_dtype(A):
    return torch.float64 if A.dtype == torch.float64 else torch.float32


def workspace_size(A, k, prm):
    dt = _check_matrix(A)
    m, n = A.shape
    nbytes = ctypes.c_size_t()
    L.check(L.load().rsvd_workspace_size(handle(A.device), dt, m, n, int(k), ctypes.byref(prm),
                                         ctypes.byref(nbytes)), "rsvd_workspace_size")
    return nbytes.value


def workspace(nbytes, device):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def rsvd(A, k, p=10, q=2, seed=0, stream_id=0, sdist="normal", precision="plain",
         compute_u=True, compute_v=True, work=None, out=None, info=None, probes=0, scheme="qr"):
    """Randomized SVD (Alg. RSVDalgorithm).  Returns (U m x k, S k, V n x k).

    U / V are None when not requested.  ``work`` (uint8 tensor) and ``out``
    (tuple U, S, V) may be passed to reuse buffers; ``info`` may be a 24-byte
    uint8 device tensor receiving the device-side record; with ``probes`` > 0
    its est_err holds the a-posteriori bound on ||A - U S V^T||_2.
    ``scheme``: "qr" (subspace iterations) or "lu" (normalized iterations).
    """
    dt = _check_matrix(A)
    m, n = A.shape
    prm = make_params(p, q, seed, stream_id, sdist, precision, probes, scheme)
    h = handle(A.device)
    nbytes = workspace_size(A, k, prm)
    if work is None or work.numel() < nbytes:
        work = workspace(nbytes, A.device)
    od = out_dtype(A)
    if out is None:
        U = torch.empty(m, k, dtype=od, device=A.device) if compute_u else None
        S = torch.empty(k, dtype=torch.float64, device=A.device)
        V = torch.empty(n, k, dtype=od, device=A.device) if compute_v else None
    else:
        U, S, V = out
    st = L.load().rsvd_run(h, dt, m, n, _ptr(A), A.stride(0), int(k), ctypes.byref(prm),
                           _ptr(U), U.stride(0) if U is not None else 0, _ptr(S),
                           _ptr(V), V.stride(0) if V is not None else 0,
                           _ptr(work), work.numel(), _ptr(info))
    L.check(st, "rsvd_run")
    return U, S, V


def rpca(A, k, center=True, retx=True, p=10, q=2, seed=0, stream_id=0, sdist="normal",
         precision="plain", work=None, info=None, probes=0, scale=False, whiten=False, loadings=False):
    """Randomized PCA (Alg. RPCAalgorithm) with implicit centring and, with
    ``scale=True``, implicit scaling to unit variance (rpca_run_ex).

    Returns a dict: rotation (n x k), eigvals, sdev, x (m x k or None),
    center, scale, total_var (0-d f64 tensor), and with ``whiten`` /
    ``loadings`` the whitened components x_white (m x k) / loadings (n x k).
    """
    dt = _check_matrix(A)
    m, n = A.shape
    prm = make_params(p, q, seed, stream_id, sdist, precision, probes)
    h = handle(A.device)
    nbytes = workspace_size(A, k, prm)
    if work is None or work.numel() < nbytes:
        work = workspace(nbytes, A.device)
    od = out_dtype(A)
    dev = A.device
    rot = torch.empty(n, k, dtype=od, device=dev)
    ev = torch.empty(k, dtype=torch.float64, device=dev)
    sd = torch.empty(k, dtype=torch.float64, device=dev)
    x = torch.empty(m, k, dtype=od, device=dev) if retx else None
    xw = torch.empty(m, k, dtype=od, device=dev) if whiten else None
    ld = torch.empty(n, k, dtype=od, device=dev) if loadings else None
    ctr = torch.empty(n, dtype=od, device=dev)
    scl = torch.empty(n, dtype=od, device=dev)
    tv = torch.empty((), dtype=torch.float64, device=dev)
    opt = L.RpcaOptions(int(bool(center)), int(bool(scale)))
    out = L.RpcaOutputs(_ptr(rot), rot.stride(0), _ptr(ev), _ptr(sd), _ptr(x), x.stride(0) if retx else 0,
                        _ptr(xw), xw.stride(0) if whiten else 0, _ptr(ld), ld.stride(0) if loadings else 0,
                        _ptr(ctr), _ptr(scl), _ptr(tv))
    st = L.load().rpca_run_ex(h, dt, m, n, _ptr(A), A.stride(0), int(k), ctypes.byref(opt), ctypes.byref(prm),
                              ctypes.byref(out), _ptr(work), work.numel(), _ptr(info))
    L.check(st, "rpca_run_ex")
    res = dict(rotation=rot, eigvals=ev, sdev=sd, x=x, center=ctr, scale=scl, total_var=tv)
    if whiten:
        res["x_white"] = xw
    if loadings:
        res["loadings"] = ld
    return res


def rpca_predict(A_new, res, center=True, scale=True):
    """Principal components of new rows with a fitted rpca result ``res``
    (rpca_predict): ((A_new - 1 center^T) / scale) rotation."""
    dt = _check_matrix(A_new)
    m, n = A_new.shape
    rot = res["rotation"]
    k = rot.shape[1]
    nbytes = ctypes.c_size_t()
    h = handle(A_new.device)
    L.check(L.load().rpca_predict_workspace_size(h, dt, m, n, k, ctypes.byref(nbytes)),
            "rpca_predict_workspace_size")
    work = workspace(nbytes.value, A_new.device)
    x = torch.empty(m, k, dtype=out_dtype(A_new), device=A_new.device)
    L.check(L.load().rpca_predict(h, dt, m, n, _ptr(A_new), A_new.stride(0), k, _ptr(rot), rot.stride(0),
                                  _ptr(res["center"]) if center else None, _ptr(res["scale"]) if scale else None,
                                  _ptr(x), x.stride(0), _ptr(work), work.numel()), "rpca_predict")
    return x


def rpca_summary(res):
    """Sec. 4.3's summary of a fitted rpca result (host arithmetic on the k
    returned values): standard deviations, proportion of variance
    eigvals / total_var, and its cumulative sum."""
    ev = res["eigvals"].double().cpu()
    prop = ev / float(res["total_var"])
    return dict(sdev=res["sdev"].double().cpu(), proportion=prop, cumulative=torch.cumsum(prop, 0))


def rrpca(A, lam=None, maxiter=50, tol=1e-5, p=10, q=2, seed=0, rho=1.6, k_max=0, work=None):
    """Robust PCA (Alg. rpca, rrpca_run): A = L + S.  Synchronises the stream
    (the method reads two scalars per iteration).  Returns dict(L, S,
    iterations, rank, k, residual, lam)."""
    dt = _check_matrix(A)
    m, n = A.shape
    prm = make_params(p, q, seed)
    opt = L.RrpcaOptions()
    L.load().rrpca_default_options(ctypes.byref(opt))
    opt.lam = 0.0 if lam is None else float(lam)
    opt.maxiter, opt.tol, opt.rho, opt.k_max = int(maxiter), float(tol), float(rho), int(k_max)
    h = handle(A.device)
    nbytes = ctypes.c_size_t()
    L.check(L.load().rrpca_workspace_size(h, dt, m, n, ctypes.byref(opt), ctypes.byref(prm), ctypes.byref(nbytes)),
            "rrpca_workspace_size")
    if work is None or work.numel() < nbytes.value:
        work = workspace(nbytes.value, A.device)
    Lo = torch.empty(m, n, dtype=out_dtype(A), device=A.device)
    So = torch.empty(m, n, dtype=out_dtype(A), device=A.device)
    res = L.RrpcaResult()
    L.check(L.load().rrpca_run(h, dt, m, n, _ptr(A), A.stride(0), ctypes.byref(opt), ctypes.byref(prm), _ptr(Lo),
                               Lo.stride(0), _ptr(So), So.stride(0), _ptr(work), work.numel(), ctypes.byref(res)),
            "rrpca_run")
    return dict(L=Lo, S=So, iterations=res.iterations, rank=res.rank, k=res.k, residual=res.residual,
                lam=res.lam)


def _id_work(dt, A, k, prm, cur):
    nbytes = ctypes.c_size_t()
    L.check(L.load().rid_workspace_size(handle(A.device), dt, A.shape[0], A.shape[1], int(k), ctypes.byref(prm),
                                        int(cur), ctypes.byref(nbytes)), "rid_workspace_size")
    return workspace(nbytes.value, A.device)


def rid(A, k, p=10, q=0, seed=0, stream_id=0, sdist="normal", idx_only=False):
    """Randomized column interpolative decomposition (Alg. rid, rid_run):
    returns dict(J (k column indices), C (m x k) and Z (k x n), None with
    idx_only) with A ~ C Z."""
    dt = _check_matrix(A)
    m, n = A.shape
    prm = make_params(p, q, seed, stream_id, sdist)
    work = _id_work(dt, A, k, prm, 0)
    od = out_dtype(A)
    J = torch.empty(k, dtype=torch.int32, device=A.device)
    C = None if idx_only else torch.empty(m, k, dtype=od, device=A.device)
    Z = None if idx_only else torch.empty(k, n, dtype=od, device=A.device)
    L.check(L.load().rid_run(handle(A.device), dt, m, n, _ptr(A), A.stride(0), int(k), ctypes.byref(prm), _ptr(J),
                             _ptr(C), k, _ptr(Z), n, _ptr(work), work.numel()), "rid_run")
    return dict(J=J, C=C, Z=Z)


def rcur(A, k, p=10, q=0, seed=0, stream_id=0, sdist="normal"):
    """Randomized CUR decomposition (Alg. rcur, rcur_run): dict(C m x k,
    U k x k, R k x n, J column indices, I row indices) with A ~ C U R."""
    dt = _check_matrix(A)
    m, n = A.shape
    prm = make_params(p, q, seed, stream_id, sdist)
    work = _id_work(dt, A, k, prm, 1)
    od = out_dtype(A)
    dev = A.device
    J = torch.empty(k, dtype=torch.int32, device=dev)
    I = torch.empty(k, dtype=torch.int32, device=dev)
    C = torch.empty(m, k, dtype=od, device=dev)
    U = torch.empty(k, k, dtype=od, device=dev)
    R = torch.empty(k, n, dtype=od, device=dev)
    L.check(L.load().rcur_run(handle(dev), dt, m, n, _ptr(A), A.stride(0), int(k), ctypes.byref(prm), _ptr(J),
                              _ptr(I), _ptr(C), k, _ptr(U), k, _ptr(R), n, _ptr(work), work.numel()), "rcur_run")
    return dict(C=C, U=U, R=R, J=J, I=I)


_DESC_DTYPE = None


def _desc_dtype():
    import numpy as np
    names = ["A", "lda", "m", "n", "k", "stream_id", "U", "ldu", "S", "V", "ldv", "info", "features", "q", "p"]
    fmts = ["<u8", "<i8", "<i8", "<i8", "<i4", "<u4", "<u8", "<i8", "<u8", "<u8", "<i8", "<u8", "<u8", "<i4", "<i4"]
    offs = [getattr(L.BatchDesc, f).offset for f in names]
    return np.dtype({"names": names, "formats": fmts, "offsets": offs, "itemsize": ctypes.sizeof(L.BatchDesc)})


class _Views:
    """Per-matrix views into a flat output buffer, made on access."""

    def __init__(self, flat, offs, rows, cols):
        self.flat, self.offs, self.rows, self.cols = flat, offs, rows, cols

    def __len__(self):
        return len(self.offs) - 1

    def __getitem__(self, b):
        v = self.flat[int(self.offs[b]):int(self.offs[b + 1])]
        return v if self.rows is None else v.view(int(self.rows[b]), int(self.cols[b]))

    def __iter__(self):
        return (self[b] for b in range(len(self)))


class _Nones:
    def __init__(self, n):
        self.n = n

    def __len__(self):
        return self.n

    def __getitem__(self, b):
        if not -self.n <= b < self.n:
            raise IndexError(b)
        return None

    def __iter__(self):
        return iter([None] * self.n)


class Batch:
    """A ragged batch of randomized SVDs run as grouped launches (rsvd_batch_*).

    ``As``: list of 2-D row-major tensors on one device, one dtype (views into
    one buffer are fine).  ``ks``: target rank per matrix.  ``stream_ids``:
    Omega stream per matrix (default: the matrix index).  Outputs live in
    ``U``, ``S``, ``V`` (lists of views into three flat buffers) after
    ``run()`` and the stream completing.  ``graph=True`` replays one captured
    HIP graph per run; ``stamps=True`` records device-clock stamps per matrix.
    ``qs`` / ``ps``: per-matrix q and p (lists) instead of ``q`` / ``p``.
    ``features=True``: run only the q = 0 sketches and fill ``features``
    (count x 131) with the selector inputs.  ``work``: optional uint8 device
    tensor reused as the workspace when large enough (owned by this batch
    while it is alive).  ``probes`` > 0: each info record's est_err receives
    the a-posteriori error bound (needs ``infos=True`` to be read).
    ``learned=True`` (rsvd_batch_create_learned): q chosen per matrix on the
    device by the selector network ``theta`` (a device f32 tensor of
    MLP_PARAMS values, or None for q = LEARNED_FALLBACK_Q everywhere) with
    threshold ``tau``, every solve with oversampling ``p`` (<= LEARNED_PMAX)
    and starting from its q = 0 sketch; ``q``, ``qs``, ``ps`` are not used and
    ``choices()`` returns the q of the last run.  ``chunked=True``
    (RSVD_BATCH_CHUNKED): each size class runs as 4 chunks of about equal
    work one after another, so a solve spans about a quarter of the batch.
    """

    def __init__(self, As, ks, p=10, q=2, seed=0, stream_ids=None, sdist="normal", precision="plain",
                 compute_u=True, compute_v=True, graph=True, stamps=False, infos=False, qs=None, ps=None,
                 features=False, work=None, probes=0, learned=False, theta=None, tau=0.8, chunked=False):
        global _DESC_DTYPE
        if _DESC_DTYPE is None:
            _DESC_DTYPE = _desc_dtype()
        if len(As) == 0 or len(As) != len(ks):
            raise ValueError("As and ks must be non-empty lists of equal length")
        dts = {_check_matrix(A) for A in As}
        if len(dts) != 1:
            raise ValueError("every matrix of a batch must have the same dtype")
        self.dtype = dts.pop()
        dev = As[0].device
        self.device = dev
        self.count = len(As)
        od = out_dtype(As[0])
        shapes = [(int(A.shape[0]), int(A.shape[1]), int(k)) for A, k in zip(As, ks)]
        if features:
            compute_u = compute_v = False
        self.features = (torch.zeros(self.count, L.MLP_INPUTS, dtype=torch.float32, device=dev)
                         if features else None)
        import numpy as np
        sh = np.array(shapes, dtype=np.int64).reshape(-1, 3)
        m_, n_, k_ = sh[:, 0], sh[:, 1], sh[:, 2]
        u_off = np.concatenate([[0], np.cumsum(m_ * k_)])
        v_off = np.concatenate([[0], np.cumsum(n_ * k_)])
        s_off = np.concatenate([[0], np.cumsum(k_)])
        self.u_flat = torch.empty(max(int(u_off[-1]), 1), dtype=od, device=dev) if compute_u else None
        self.v_flat = torch.empty(max(int(v_off[-1]), 1), dtype=od, device=dev) if compute_v else None
        self.s_flat = torch.empty(int(s_off[-1]), dtype=torch.float64, device=dev)
        self.info = (torch.zeros(self.count, ctypes.sizeof(L.Info), dtype=torch.uint8, device=dev)
                     if infos else None)
        self.U = _Views(self.u_flat, u_off, m_, k_) if compute_u else _Nones(self.count)
        self.V = _Views(self.v_flat, v_off, n_, k_) if compute_v else _Nones(self.count)
        self.S = _Views(self.s_flat, s_off, None, k_)
        # descriptors filled column by column (the layout of rsvd_batch_desc)
        d = np.zeros(self.count, dtype=_DESC_DTYPE)
        d["A"] = [A.data_ptr() for A in As]
        d["lda"] = [A.stride(0) for A in As]
        d["m"], d["n"], d["k"] = m_, n_, k_
        d["stream_id"] = np.arange(self.count) if stream_ids is None else np.asarray(stream_ids)
        esz = 4 if od == torch.float32 else 8
        if compute_u:
            d["U"] = self.u_flat.data_ptr() + u_off[:-1] * esz
            d["ldu"] = k_
        if compute_v:
            d["V"] = self.v_flat.data_ptr() + v_off[:-1] * esz
            d["ldv"] = k_
        d["S"] = self.s_flat.data_ptr() + s_off[:-1] * 8
        if infos:
            d["info"] = self.info.data_ptr() + np.arange(self.count) * ctypes.sizeof(L.Info)
        if features:
            d["features"] = self.features.data_ptr() + np.arange(self.count) * (L.MLP_INPUTS * 4)
        d["q"] = np.asarray(qs) if qs is not None else q
        d["p"] = np.asarray(ps) if ps is not None else p
        self._desc = d
        descs = d.ctypes.data_as(ctypes.c_void_p)
        self._As = list(As)            # keep the inputs alive as long as the batch
        prm = make_params(p, q, seed, 0, sdist, precision, 0 if features else probes)
        flags = (L.BATCH_GRAPH if graph else 0) | (L.BATCH_STAMPS if stamps else 0)
        flags |= (L.BATCH_FEATURES if features else 0) | (L.BATCH_OWN_QP if (qs is not None or ps is not None) else 0)
        flags |= L.BATCH_CHUNKED if chunked else 0
        self._lib = L.load()
        self._h = handle(dev)
        self._b = ctypes.c_void_p()
        nbytes = ctypes.c_size_t()
        self.learned = bool(learned)
        if self.learned:
            if features or qs is not None or ps is not None:
                raise ValueError("a learned batch chooses q itself and computes its own features")
            self._theta = theta            # read by every run: keep it alive
            flags &= L.BATCH_GRAPH | L.BATCH_STAMPS
            L.check(self._lib.rsvd_batch_create_learned(self._h, self.dtype, self.count, descs, ctypes.byref(prm),
                                                        _ptr(theta), float(tau), flags, ctypes.byref(self._b),
                                                        ctypes.byref(nbytes)), "rsvd_batch_create_learned")
        else:
            L.check(self._lib.rsvd_batch_create(self._h, self.dtype, self.count, descs, ctypes.byref(prm), flags,
                                                ctypes.byref(self._b), ctypes.byref(nbytes)), "rsvd_batch_create")
        self.work_bytes = nbytes.value
        # a caller-provided workspace (uint8 tensor) is used when large enough;
        # it must not be shared with another live batch
        self.work = work if (work is not None and work.numel() >= nbytes.value) else workspace(nbytes.value, dev)
        L.check(self._lib.rsvd_batch_bind(self._b, _ptr(self.work), self.work.numel()), "rsvd_batch_bind")

    def run(self):
        handle(self.device)            # follow torch's current stream
        L.check(self._lib.rsvd_batch_run(self._b), "rsvd_batch_run")

    def stamps(self):
        """(count x 2 int64 numpy array of device-clock stamps, ticks per second)."""
        import numpy as np
        out = np.zeros((self.count, 2), dtype=np.uint64)
        hz = ctypes.c_double()
        L.check(self._lib.rsvd_batch_stamps(self._b, out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(hz)),
                "rsvd_batch_stamps")
        return out.astype(np.int64), hz.value

    def choices(self):
        """Learned batches: the q chosen for each matrix by the last run (synchronises)."""
        import numpy as np
        out = np.zeros(self.count, dtype=np.int32)
        L.check(self._lib.rsvd_batch_choices(self._b, out.ctypes.data_as(ctypes.c_void_p)), "rsvd_batch_choices")
        return out

    def infos(self):
        """Decode the per-matrix info records (synchronises)."""
        torch.cuda.synchronize(self.device)
        raw = self.info.cpu().numpy()
        return [L.Info.from_buffer_copy(raw[b].tobytes()) for b in range(self.count)]

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            self._lib.rsvd_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def new_info(device):
    return torch.zeros(ctypes.sizeof(L.Info), dtype=torch.uint8, device=device)


def sync_info(info):
    """Synchronise and decode a device info record; returns (status, Info)."""
    host = L.Info()
    st = L.load().rsvd_sync_info(handle(info.device), _ptr(info), ctypes.byref(host))
    return st, host


def profile_enable(enable=True, device=None):
    """Bracket every product with A by HIP events on the library's stream."""
    L.check(L.load().rsvd_profile_enable(handle(device), int(bool(enable))), "rsvd_profile_enable")


def profile_collect(device=None):
    """Synchronise and return {kind: dict(count, total_ms, flops, bytes)}."""
    stats = (L.KernelStat * L.PROFILE_KINDS)()
    L.check(L.load().rsvd_profile_collect(handle(device), stats), "rsvd_profile_collect")
    return {name: dict(count=s.count, total_ms=s.total_ms, flops=s.flops, bytes=s.bytes)
            for name, s in zip(L.PROFILE_NAMES, stats)}


# ---------------------------------------------------------------- building blocks

def philox_words(n, groups, seed, stream_id=0, device="cuda"):
    out = torch.empty(n, 4 * groups, dtype=torch.int32, device=device)
    L.check(L.load().rsvd_philox_words(handle(device), n, groups, seed, stream_id, _ptr(out)),
            "rsvd_philox_words")
    return out


def test_matrix(n, l, seed, stream_id=0, sdist="normal", dtype=torch.float64, device="cuda"):
    out = torch.empty(n, l, dtype=dtype, device=device)
    dt = L.RSVD_F64 if dtype == torch.float64 else L.RSVD_F32
    L.check(L.load().rsvd_test_matrix(handle(device), dt, n, l, seed, stream_id, L.SDIST[sdist],
                                      _ptr(out), out.stride(0)), "rsvd_test_matrix")
    return out


def _block_ws(dt, m, n, c, device):
    nbytes = ctypes.c_size_t()
    L.check(L.load().rsvd_block_workspace_size(handle(device), dt, m, n, c, ctypes.byref(nbytes)),
            "rsvd_block_workspace_size")
    return workspace(nbytes.value, device)


def gemm_nn(A, X, arith="storage", splits=1):
    """Y = A X with the library's product kernel (arith: storage, bf16, split).

    splits: chunks of the K-reduction (1..4), or 0 for the split rsvd_run
    takes at this shape."""
    dt = _check_matrix(A)
    m, K = A.shape
    c = X.shape[1]
    Y = torch.empty(m, c, dtype=out_dtype(A), device=A.device)
    work = _block_ws(dt, m, K, c, A.device)
    L.check(L.load().rsvd_gemm_nn(handle(A.device), dt, L.ARITH[arith], m, K, c, _ptr(A), A.stride(0), _ptr(X),
                                  X.stride(0), _ptr(Y), Y.stride(0), int(splits), _ptr(work),
                                  work.numel() if work is not None else 0), "rsvd_gemm_nn")
    return Y


def gemm_tn(A, Q, arith="storage"):
    """Z = A^T Q with the library's split-K product kernel (arith: storage, bf16, split)."""
    dt = _check_matrix(A)
    m, n = A.shape
    c = Q.shape[1]
    Z = torch.empty(n, c, dtype=out_dtype(A), device=A.device)
    work = _block_ws(dt, m, n, c, A.device)
    L.check(L.load().rsvd_gemm_tn(handle(A.device), dt, L.ARITH[arith], m, n, c, _ptr(A), A.stride(0), _ptr(Q),
                                  Q.stride(0), _ptr(Z), Z.stride(0), _ptr(work), work.numel()),
            "rsvd_gemm_tn")
    return Z


def orthonormalize(Y):
    """In-place CholeskyQR2 of Y (m x c); returns (Y, R, flags tensor)."""
    dt = _check_matrix(Y)
    m, c = Y.shape
    R = torch.empty(c, c, dtype=torch.float64, device=Y.device)
    flags = torch.zeros(1, dtype=torch.int32, device=Y.device)
    work = _block_ws(dt, m, m, c, Y.device)
    L.check(L.load().rsvd_orthonormalize(handle(Y.device), dt, m, c, _ptr(Y), Y.stride(0), _ptr(R),
                                         _ptr(flags), _ptr(work), work.numel()), "rsvd_orthonormalize")
    return Y, R, flags


def lu_normalize(Y):
    """In-place pivoted LU normalisation of Y (m x c): Y <- L; returns (Y, U,
    piv, flags tensor)."""
    dt = _check_matrix(Y)
    m, c = Y.shape
    U = torch.empty(c, c, dtype=torch.float64, device=Y.device)
    piv = torch.empty(c, dtype=torch.int32, device=Y.device)
    flags = torch.zeros(1, dtype=torch.int32, device=Y.device)
    work = _block_ws(dt, m, m, c, Y.device)
    L.check(L.load().rsvd_lu_normalize(handle(Y.device), dt, m, c, _ptr(Y), Y.stride(0), _ptr(piv), _ptr(U),
                                       _ptr(flags), _ptr(work), work.numel()), "rsvd_lu_normalize")
    return Y, U, piv, flags


def small_svd(R):
    """R (c x c, f64) = W diag(s) J^T via the one-workgroup Jacobi kernel."""
    c = R.shape[0]
    R = R.contiguous()
    s = torch.empty(c, dtype=torch.float64, device=R.device)
    W = torch.empty(c, c, dtype=torch.float64, device=R.device)
    J = torch.empty(c, c, dtype=torch.float64, device=R.device)
    flags = torch.zeros(1, dtype=torch.int32, device=R.device)
    work = _block_ws(L.RSVD_F64, c, c, c, R.device)
    L.check(L.load().rsvd_small_svd(handle(R.device), c, _ptr(R), _ptr(s), _ptr(W), _ptr(J), _ptr(flags),
                                    _ptr(work), work.numel()), "rsvd_small_svd")
    return s, W, J, flags


# ---------------------------------------------------------------- selector network

def mlp_init(seed=0, device="cuda"):
    """Fresh selector-network parameters (f32 vector of MLP_PARAMS values)."""
    theta = torch.empty(L.MLP_PARAMS, dtype=torch.float32, device=device)
    L.check(L.load().rsvd_mlp_init(handle(device), _ptr(theta), int(seed)), "rsvd_mlp_init")
    return theta


def _mlp_x(X):
    if X.dtype != torch.float32 or X.dim() != 2 or X.shape[1] != L.MLP_INPUTS or not X.is_contiguous():
        raise ValueError("features must be a contiguous float32 tensor of shape (batch, 131)")
    return X


def mlp_forward(theta, X):
    """(prob batch x 15, class batch) of the selector network."""
    X = _mlp_x(X)
    B = X.shape[0]
    prob = torch.empty(B, L.MLP_CLASSES, dtype=torch.float32, device=X.device)
    cls = torch.empty(B, dtype=torch.int32, device=X.device)
    L.check(L.load().rsvd_mlp_forward(handle(X.device), _ptr(theta), B, _ptr(X), _ptr(prob), _ptr(cls)),
            "rsvd_mlp_forward")
    return prob, cls


class MlpTrainer:
    """Adam training of the selector network through rsvd_mlp_train_step."""

    def __init__(self, theta, lr=1e-3):
        self.theta = theta
        self.m = torch.zeros_like(theta)
        self.v = torch.zeros_like(theta)
        self.step_no = 0
        self.lr = float(lr)
        self.loss = torch.zeros(1, dtype=torch.float32, device=theta.device)
        self.grad = torch.zeros_like(theta)
        self._work = None

    def _ws(self, B):
        nbytes = ctypes.c_size_t()
        L.check(L.load().rsvd_mlp_workspace_size(B, ctypes.byref(nbytes)), "rsvd_mlp_workspace_size")
        if self._work is None or self._work.numel() < nbytes.value:
            self._work = workspace(nbytes.value, self.theta.device)
        return self._work

    def step(self, X, y, update=True):
        """One step on (X batch x 131, y batch int32); returns the loss tensor."""
        X = _mlp_x(X)
        y = y.to(torch.int32).contiguous()
        B = X.shape[0]
        work = self._ws(B)
        if update:
            self.step_no += 1
        L.check(L.load().rsvd_mlp_train_step(handle(X.device), _ptr(self.theta), _ptr(self.m), _ptr(self.v),
                                             self.step_no if update else 0, self.lr, B, _ptr(X), _ptr(y),
                                             _ptr(self.grad), _ptr(self.loss), _ptr(work), work.numel()),
                "rsvd_mlp_train_step")
        return self.loss


_scratch_ws = {}


def _scratch(nbytes, device):
    """Per-device scratch workspace reused by synchronous calls (select)."""
    key = str(device)
    t = _scratch_ws.get(key)
    if t is None or t.numel() < nbytes:
        _scratch_ws[key] = t = workspace(nbytes, device)
    return t


def select(As, ks, theta, seed=0, stream_ids=None, sdist="normal", precision="plain", tau=0.0):
    """Learned (q, p) per matrix (rsvd_select): returns (qs, ps, features).
    tau <= 0: the network's most probable class; otherwise the cheapest class
    whose dominated probability mass reaches tau."""
    import numpy as np
    dts = {_check_matrix(A) for A in As}
    if len(dts) != 1:
        raise ValueError("every matrix must have the same dtype")
    dt = dts.pop()
    dev = As[0].device
    n = len(As)
    global _DESC_DTYPE
    if _DESC_DTYPE is None:
        _DESC_DTYPE = _desc_dtype()
    d = np.zeros(n, dtype=_DESC_DTYPE)
    d["A"] = [A.data_ptr() for A in As]
    d["lda"] = [A.stride(0) for A in As]
    d["m"] = [A.shape[0] for A in As]
    d["n"] = [A.shape[1] for A in As]
    d["k"] = np.asarray(ks)
    d["stream_id"] = np.arange(n) if stream_ids is None else np.asarray(stream_ids)
    descs = d.ctypes.data_as(ctypes.c_void_p)
    prm = make_params(10, 0, seed, 0, sdist, precision)
    lib = L.load()
    h = handle(dev)
    nbytes = ctypes.c_size_t()
    L.check(lib.rsvd_select_workspace_size(h, dt, n, descs, ctypes.byref(prm), ctypes.byref(nbytes)),
            "rsvd_select_workspace_size")
    work = _scratch(nbytes.value, dev)
    feats = torch.empty(n, L.MLP_INPUTS, dtype=torch.float32, device=dev)
    qs = np.zeros(n, dtype=np.int32)
    ps = np.zeros(n, dtype=np.int32)
    L.check(lib.rsvd_select(h, dt, n, descs, ctypes.byref(prm), _ptr(theta), float(tau),
                            qs.ctypes.data_as(ctypes.c_void_p), ps.ctypes.data_as(ctypes.c_void_p),
                            _ptr(feats), _ptr(work), work.numel()), "rsvd_select")
    return qs, ps, feats
