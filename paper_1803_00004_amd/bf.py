"""ctypes binding of libbf.so (the C ABI of include/bf.h).

Argument marshalling only: every step of the filter runs in the library's HIP
kernels.  torch tensors are used for device memory and streams.  The library
must have been built (paper_1803_00004_amd/build.py); importing this module
without it raises, there is no fallback.
"""
import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libbf.so")

BF_OK, BF_ERR_INVALID_ARG, BF_ERR_OUT_OF_MEMORY, BF_ERR_DEVICE, BF_ERR_UNSUPPORTED = range(5)
BF_KERNEL_GAUSSIAN = 0
BF_KERNEL_EXPONENTIAL = 1
KERNELS = {"gaussian": BF_KERNEL_GAUSSIAN, "exponential": BF_KERNEL_EXPONENTIAL}
BF_IN_F32, BF_IN_U8 = 0, 1
BF_PREC_PLAIN, BF_PREC_REDUCED = 0, 1
BF_FLAG_HOST_ONLY = 0x1
BF_FLAG_DIRECT = 0x2
BF_FLAG_DIRECT_AUTO = 0x4
BF_FLAG_RANGE_BOX = 0x8
BF_FLAG_LEVEL_FOLD = 0x10

EXPORTED = [
    "bf_plan_create", "bf_plan_create_tabulated", "bf_plan_destroy", "bf_workspace_size", "bf_filter", "bf_filter_ws",
    "bf_filter_parts", "bf_batch_workspace_size", "bf_filter_batch", "bf_plan_query",
    "bf_image_geometry", "bf_image_lookup_kernel", "bf_plan_range_terms", "bf_plan_spatial_kernel", "bf_plan_taps", "bf_plan_spatial_groups",
    "bf_profile_enable", "bf_profile_read", "bf_status_string", "bf_version",
    "bf_server_create", "bf_server_destroy", "bf_server_submit", "bf_server_poll", "bf_server_pending",
    "bf_server_stats", "bf_autotune", "bf_tuning_set", "bf_autotune_clear",
    "bf_precompute_size", "bf_precompute", "bf_precomputed_compatible", "bf_filter_precomputed",
    "bf_filter_noalloc", "bf_batch_set_fused",
]
NOALLOC_SCRATCH_BYTES = 256 << 20


class BFError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__("%s failed: %s" % (what, status_string(status)))


class _Terms(ctypes.Structure):
    _fields_ = [("n_range", ctypes.c_int), ("n_spatial", ctypes.c_int)]


class _Opts(ctypes.Structure):
    _fields_ = [("in_dtype", ctypes.c_int), ("precision", ctypes.c_int), ("eps", ctypes.c_double),
                ("span", ctypes.c_double), ("tile", ctypes.c_int), ("flags", ctypes.c_uint)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("radius", ctypes.c_int), ("n_range", ctypes.c_int), ("n_spatial", ctypes.c_int),
                ("n_taps", ctypes.c_int), ("n_tap_rows", ctypes.c_int), ("n_tap_cols", ctypes.c_int),
                ("n_images", ctypes.c_int), ("tile", ctypes.c_int), ("sat_shift", ctypes.c_int),
                ("T_s", ctypes.c_double), ("T_r", ctypes.c_double), ("T", ctypes.c_double),
                ("den_floor", ctypes.c_double), ("n_quads", ctypes.c_int), ("n_single", ctypes.c_int),
                ("lookup_kernel", ctypes.c_int), ("direct", ctypes.c_int), ("range_box", ctypes.c_int),
                ("box_levels", ctypes.c_int), ("box_tile", ctypes.c_int), ("reduced", ctypes.c_int),
                ("level_fold", ctypes.c_int), ("lds_pitch", ctypes.c_int), ("lds_double_buffered", ctypes.c_int),
                ("lattice", ctypes.c_int), ("lattice_step", ctypes.c_int), ("default_lookup", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def lib():
    """Load libbf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libbf.so is not built: run python paper_1803_00004_amd/build.py "
                              "(or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
        ip, dp = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
        L.bf_plan_create.argtypes = [ctypes.POINTER(vp), i, i, d, d, i, _Terms, ctypes.POINTER(_Opts)]
        L.bf_plan_create_tabulated.argtypes = [ctypes.POINTER(vp), dp, i, dp, i, d, _Terms, ctypes.POINTER(_Opts)]
        L.bf_plan_destroy.argtypes = [vp]
        L.bf_workspace_size.argtypes = [vp, i, i, ctypes.POINTER(sz)]
        L.bf_filter.argtypes = [vp, vp, vp, i, i, vp]
        L.bf_filter_ws.argtypes = [vp, vp, vp, i, i, vp, sz, vp]
        L.bf_filter_noalloc.argtypes = [vp, vp, vp, i, i, vp]
        L.bf_batch_set_fused.argtypes = [i]
        L.bf_filter_parts.argtypes = [vp, vp, vp, vp, vp, i, i, vp, sz, vp]
        L.bf_batch_workspace_size.argtypes = [ctypes.POINTER(vp), i, ip, ip, ctypes.POINTER(sz)]
        L.bf_filter_batch.argtypes = [ctypes.POINTER(vp), i, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                      ip, ip, vp, sz, vp]
        L.bf_plan_query.argtypes = [vp, ctypes.POINTER(PlanInfo)]
        L.bf_image_geometry.argtypes = [vp, i, i, ip, ip, ctypes.POINTER(sz)]
        L.bf_image_lookup_kernel.argtypes = [vp, i, i, ip]
        L.bf_plan_range_terms.argtypes = [vp, ip, dp, dp, i]
        L.bf_plan_spatial_kernel.argtypes = [vp, dp, i]
        L.bf_plan_taps.argtypes = [vp, ip, ip, dp, i]
        L.bf_plan_spatial_groups.argtypes = [vp, ip, ip, i]
        L.bf_autotune.argtypes = [vp, i, i, i, vp, ip]
        L.bf_tuning_set.argtypes = [vp, i, i, i, i, i]
        L.bf_autotune_clear.argtypes = []
        L.bf_precompute_size.argtypes = [vp, i, i, ctypes.POINTER(sz)]
        L.bf_precompute.argtypes = [vp, vp, i, i, vp, sz, vp]
        L.bf_precomputed_compatible.argtypes = [vp, vp]
        L.bf_filter_precomputed.argtypes = [vp, vp, vp, vp, i, i, vp, sz, vp]
        L.bf_server_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(_ServerOpts)]
        L.bf_server_destroy.argtypes = [vp]
        L.bf_server_submit.argtypes = [vp, vp, vp, vp, i, i, ctypes.c_ulonglong, d]
        L.bf_server_poll.argtypes = [vp, d, ctypes.POINTER(Completion), i, ip]
        L.bf_server_pending.argtypes = [vp, ip, ip]
        L.bf_server_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
        L.bf_version.argtypes = []
        L.bf_profile_enable.argtypes = [i]
        L.bf_profile_read.argtypes = [dp, ip]
        L.bf_status_string.argtypes = [i]
        L.bf_status_string.restype = ctypes.c_char_p
        L.bf_version.restype = ctypes.c_char_p
        for name in EXPORTED:
            if name not in ("bf_status_string", "bf_version"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def profile_enable(on=True):
    _check(lib().bf_profile_enable(1 if on else 0), "bf_profile_enable")


def profile_read():
    """(ms[2], launches[2]) summed since the last read: [tables kernel, lookup kernel]."""
    ms = (ctypes.c_double * 2)()
    n = (ctypes.c_int * 2)()
    _check(lib().bf_profile_read(ms, n), "bf_profile_read")
    return list(ms), list(n)


def status_string(s):
    return lib().bf_status_string(int(s)).decode()


def _check(status, what):
    if status != BF_OK:
        raise BFError(status, what)


def _stream_handle(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """A filter plan: both kernel expansions fitted (FP64, host) and uploaded."""

    def __init__(self, sigma_s, sigma_r, radius=0, n_range=8, n_spatial=4, dtype="f32",
                 precision="plain", eps=0.0, span=0.0, tile=0, host_only=False, direct=False,
                 kernel_s="gaussian", kernel_r="gaussian", range_box=False, level_fold=False, tables=None):
        """direct: False (N-term expansion), True (direct summation of Eq. BF,
        BF_FLAG_DIRECT) or "auto" (direct where its cost model is lower).
        kernel_s / kernel_r: "gaussian" or "exponential" (bf_kernel_t).
        tables: (K_s weights (2r+1) x (2r+1), K_r samples, sample step) for
        bf_plan_create_tabulated (sigma_s, sigma_r, radius, kernel_s / _r and
        eps are then unused); see Plan.tabulated.
        range_box: the paper's own 8-bit regime, T = T_r with the range box
        (BF_FLAG_RANGE_BOX; dtype "u8" only).
        level_fold: 8-bit input, the default regime with the range terms folded
        per output level (BF_FLAG_LEVEL_FOLD; dtype "u8" only)."""
        self._h = ctypes.c_void_p()
        flags = BF_FLAG_HOST_ONLY if host_only else 0
        if direct == "auto":
            flags |= BF_FLAG_DIRECT_AUTO
        elif direct:
            flags |= BF_FLAG_DIRECT
        if range_box:
            flags |= BF_FLAG_RANGE_BOX
        if level_fold:
            flags |= BF_FLAG_LEVEL_FOLD
        opts = _Opts(BF_IN_U8 if dtype == "u8" else BF_IN_F32,
                     BF_PREC_REDUCED if precision == "reduced" else BF_PREC_PLAIN,
                     float(eps), float(span), int(tile), flags)
        if tables is not None:
            ks = np.ascontiguousarray(tables[0], dtype=np.float64)
            kr = np.ascontiguousarray(tables[1], dtype=np.float64)
            if ks.ndim != 2 or ks.shape[0] != ks.shape[1] or ks.shape[0] % 2 != 1 or kr.ndim != 1:
                raise ValueError("tables: K_s must be (2r+1) x (2r+1), K_r one-dimensional")
            dp = ctypes.POINTER(ctypes.c_double)
            st = lib().bf_plan_create_tabulated(ctypes.byref(self._h), ks.ctypes.data_as(dp),
                                                (ks.shape[0] - 1) // 2, kr.ctypes.data_as(dp), len(kr),
                                                float(tables[2]), _Terms(int(n_range), int(n_spatial)),
                                                ctypes.byref(opts))
            _check(st, "bf_plan_create_tabulated")
        else:
            st = lib().bf_plan_create(ctypes.byref(self._h), KERNELS[kernel_s], KERNELS[kernel_r],
                                      float(sigma_s), float(sigma_r), int(radius),
                                      _Terms(int(n_range), int(n_spatial)), ctypes.byref(opts))
            _check(st, "bf_plan_create")
        self.dtype = dtype
        self.info = self.query()

    @classmethod
    def tabulated(cls, ks, kr, kr_step, n_range=8, n_spatial=4, **kw):
        """A plan of two tabulated kernels (bf_plan_create_tabulated): K_s
        weights on the integer offsets, K_r samples at multiples of kr_step."""
        return cls(0.0, 0.0, n_range=n_range, n_spatial=n_spatial, tables=(ks, kr, kr_step), **kw)

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib().bf_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def query(self):
        info = PlanInfo()
        _check(lib().bf_plan_query(self._h, ctypes.byref(info)), "bf_plan_query")
        return info

    def range_terms(self):
        n = self.info.n_range
        k = (ctypes.c_int * n)()
        a = (ctypes.c_double * n)()
        w = (ctypes.c_double * n)()
        _check(lib().bf_plan_range_terms(self._h, k, a, w, n), "bf_plan_range_terms")
        return np.array(k[:]), np.array(a[:]), np.array(w[:])

    def spatial_kernel(self):
        r = self.info.radius
        n = (2 * r + 1) ** 2
        K = (ctypes.c_double * n)()
        _check(lib().bf_plan_spatial_kernel(self._h, K, n), "bf_plan_spatial_kernel")
        return np.array(K[:]).reshape(2 * r + 1, 2 * r + 1)

    def taps(self):
        n = self.info.n_taps
        dy, dx, w = (ctypes.c_int * n)(), (ctypes.c_int * n)(), (ctypes.c_double * n)()
        _check(lib().bf_plan_taps(self._h, dy, dx, w, n), "bf_plan_taps")
        return np.array(dy[:]), np.array(dx[:]), np.array(w[:])

    def spatial_groups(self):
        n = self.info.n_spatial
        lx, ly = (ctypes.c_int * n)(), (ctypes.c_int * n)()
        _check(lib().bf_plan_spatial_groups(self._h, lx, ly, n), "bf_plan_spatial_groups")
        return list(zip(lx[:], ly[:]))

    def geometry(self, H, W):
        """(table tile edge, fixed-point shift q, workspace bytes) for an H x W image."""
        t, q, b = ctypes.c_int(), ctypes.c_int(), ctypes.c_size_t()
        _check(lib().bf_image_geometry(self._h, int(H), int(W), ctypes.byref(t), ctypes.byref(q),
                                       ctypes.byref(b)), "bf_image_geometry")
        return t.value, q.value, b.value

    def lookup_kernel(self, H, W):
        """The lookup kernel an H x W image runs now (bf_image_lookup_kernel):
        0 per-pixel, 1 / 2 LDS tile double / single-buffered, 3 lattice, -1 none."""
        k = ctypes.c_int()
        _check(lib().bf_image_lookup_kernel(self._h, int(H), int(W), ctypes.byref(k)), "bf_image_lookup_kernel")
        return k.value

    def autotune(self, H, W, reps=5, stream=None):
        """Time the candidate tilings for H x W images and keep the fastest
        (bf_autotune); returns the chosen table tile."""
        t = ctypes.c_int()
        _check(lib().bf_autotune(self.handle, int(H), int(W), int(reps), _stream_handle(stream), ctypes.byref(t)),
               "bf_autotune")
        return t.value

    def set_tuning(self, H, W, tile, kb_single=0, ka_one=0):
        """Pin the launch shape for this plan's shape class and size bucket
        (bf_tuning_set)."""
        _check(lib().bf_tuning_set(self.handle, int(H), int(W), int(tile), int(kb_single), int(ka_one)),
               "bf_tuning_set")

    def workspace_size(self, H, W):
        b = ctypes.c_size_t()
        _check(lib().bf_workspace_size(self._h, int(H), int(W), ctypes.byref(b)), "bf_workspace_size")
        return b.value


def _image_args(plan, I):
    import torch
    if not (isinstance(I, torch.Tensor) and I.is_cuda and I.dim() == 2 and I.is_contiguous()):
        raise ValueError("I must be a contiguous 2-D CUDA tensor")
    want = torch.uint8 if plan.dtype == "u8" else torch.float32
    if I.dtype != want:
        raise ValueError("plan expects %s input" % want)
    return I.shape[0], I.shape[1]


def workspace(plan, H, W, device=None):
    """A device workspace tensor of the size bf_filter_ws needs."""
    import torch
    return torch.empty(max(1, plan.workspace_size(H, W)), dtype=torch.uint8,
                       device=device or "cuda")


def filter(plan, I, out=None, ws=None, stream=None, num=None, den=None):
    """Filter one image (torch CUDA tensor).  With ws=None the plan's own
    workspace is used (bf_filter); otherwise bf_filter_ws / bf_filter_parts."""
    import torch
    H, W = _image_args(plan, I)
    if out is None:
        out = torch.empty((H, W), dtype=torch.float32, device=I.device)
    s = _stream_handle(stream)
    if ws is None and num is None and den is None:
        st = lib().bf_filter(plan.handle, ctypes.c_void_p(I.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                             H, W, s)
        _check(st, "bf_filter")
        return out
    if ws is None:
        ws = workspace(plan, H, W, I.device)
    nump = ctypes.c_void_p(num.data_ptr()) if num is not None else None
    denp = ctypes.c_void_p(den.data_ptr()) if den is not None else None
    st = lib().bf_filter_parts(plan.handle, ctypes.c_void_p(I.data_ptr()),
                               ctypes.c_void_p(out.data_ptr()), nump, denp, H, W,
                               ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(), s)
    _check(st, "bf_filter_parts")
    return out


def filter_noalloc(plan, I, out, stream=None):
    """Filter one image into `out` with the library's per-GPU scratch array
    as workspace (bf_filter_noalloc): no device memory is allocated."""
    H, W = _image_args(plan, I)
    st = lib().bf_filter_noalloc(plan.handle, ctypes.c_void_p(I.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                 H, W, _stream_handle(stream))
    _check(st, "bf_filter_noalloc")
    return out


def set_batch_fused(on):
    """bf_batch_set_fused: run eligible batch groups as one fused launch
    (tables and lookups in one persistent kernel), process-wide."""
    _check(lib().bf_batch_set_fused(1 if on else 0), "bf_batch_set_fused")


def batch_workspace_size(plans, shapes):
    n = len(plans)
    hs = (ctypes.c_int * n)(*[int(h) for h, _ in shapes])
    wd = (ctypes.c_int * n)(*[int(w) for _, w in shapes])
    hp = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
    b = ctypes.c_size_t()
    _check(lib().bf_batch_workspace_size(hp, n, hs, wd, ctypes.byref(b)), "bf_batch_workspace_size")
    return b.value


def filter_batch(plans, images, outs=None, ws=None, stream=None):
    """Filter a list of images (torch CUDA tensors) with their plans."""
    import torch
    n = len(plans)
    shapes = [_image_args(p, I) for p, I in zip(plans, images)]
    if outs is None:
        outs = [torch.empty(s, dtype=torch.float32, device=I.device) for s, I in zip(shapes, images)]
    if ws is None:
        ws = torch.empty(max(1, batch_workspace_size(plans, shapes)), dtype=torch.uint8,
                         device=images[0].device)
    hp = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
    ip = (ctypes.c_void_p * n)(*[I.data_ptr() for I in images])
    op = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
    hs = (ctypes.c_int * n)(*[h for h, _ in shapes])
    wd = (ctypes.c_int * n)(*[w for _, w in shapes])
    st = lib().bf_filter_batch(hp, n, ip, op, hs, wd, ctypes.c_void_p(ws.data_ptr()),
                               ws.numel() * ws.element_size(), _stream_handle(stream))
    _check(st, "bf_filter_batch")
    return outs


# ---------------------------------------------------------------------------
# Serving
# ---------------------------------------------------------------------------
BF_SERVER_DRY_RUN = 1


class _ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_batch", ctypes.c_int), ("n_streams", ctypes.c_int),
                ("flags", ctypes.c_uint), ("dry_rate", ctypes.c_double)]


class Completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_ulonglong), ("status", ctypes.c_int), ("batch", ctypes.c_int),
                ("batch_size", ctypes.c_int), ("t_launch", ctypes.c_double), ("t_done", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_longlong), ("completed", ctypes.c_longlong), ("batches", ctypes.c_longlong),
                ("peak_batches_in_flight", ctypes.c_int), ("peak_requests_in_flight", ctypes.c_int),
                ("peak_arena_bytes", ctypes.c_size_t), ("arena_bytes", ctypes.c_size_t),
                ("batch_size_hist", ctypes.c_longlong * 65)]


class Server:
    """Request loop of the library (bf_server_*): queue, HBM-budget admission,
    continuous batching over several streams."""

    def __init__(self, hbm_budget=0, max_batch=0, n_streams=0, dry_run=False, dry_rate=0.0):
        o = _ServerOpts(int(hbm_budget), int(max_batch), int(n_streams),
                        BF_SERVER_DRY_RUN if dry_run else 0, float(dry_rate))
        h = ctypes.c_void_p()
        _check(lib().bf_server_create(ctypes.byref(h), ctypes.byref(o)), "bf_server_create")
        self.handle = h
        self._buf = (Completion * 256)()

    def submit(self, plan, I, out, tag, now, H=None, W=None):
        """I, out: torch tensors (or, for a dry run, H and W with any nonzero
        integers standing in for the pointers)."""
        if H is None:
            H, W = _image_args(plan, I)
            ip, op = I.data_ptr(), out.data_ptr()
        else:
            ip, op = I, out
        st = lib().bf_server_submit(self.handle, plan.handle, ctypes.c_void_p(ip), ctypes.c_void_p(op),
                                    int(H), int(W), ctypes.c_ulonglong(tag), ctypes.c_double(now))
        _check(st, "bf_server_submit")

    def poll(self, now):
        n = ctypes.c_int()
        out = []
        while True:
            _check(lib().bf_server_poll(self.handle, ctypes.c_double(now), self._buf, len(self._buf),
                                        ctypes.byref(n)), "bf_server_poll")
            out.extend(Completion.from_buffer_copy(self._buf[i]) for i in range(n.value))
            if n.value < len(self._buf):
                return out

    def pending(self):
        q, f = ctypes.c_int(), ctypes.c_int()
        _check(lib().bf_server_pending(self.handle, ctypes.byref(q), ctypes.byref(f)), "bf_server_pending")
        return q.value, f.value

    def stats(self):
        s = ServerStats()
        _check(lib().bf_server_stats(self.handle, ctypes.byref(s)), "bf_server_stats")
        return s

    def close(self):
        if self.handle:
            lib().bf_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Pre-computed tables (re-filtering one image under several plans)
# ---------------------------------------------------------------------------
def precompute(tables_plan, I, ws=None, stream=None):
    """Build the term tables of I under tables_plan (table kernel only);
    returns the workspace tensor holding them."""
    import torch
    H, W = _image_args(tables_plan, I)
    n = ctypes.c_size_t()
    _check(lib().bf_precompute_size(tables_plan.handle, H, W, ctypes.byref(n)), "bf_precompute_size")
    if ws is None:
        ws = torch.empty(max(1, n.value), dtype=torch.uint8, device=I.device)
    _check(lib().bf_precompute(tables_plan.handle, ctypes.c_void_p(I.data_ptr()), H, W,
                               ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
                               _stream_handle(stream)), "bf_precompute")
    return ws


def precomputed_compatible(tables_plan, plan):
    return lib().bf_precomputed_compatible(tables_plan.handle, plan.handle)


def filter_precomputed(tables_plan, plan, I, ws, out=None, stream=None):
    """Filter I under plan from tables built by precompute(tables_plan, I)."""
    import torch
    H, W = _image_args(plan, I)
    if out is None:
        out = torch.empty((H, W), dtype=torch.float32, device=I.device)
    _check(lib().bf_filter_precomputed(tables_plan.handle, plan.handle, ctypes.c_void_p(I.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()), H, W, ctypes.c_void_p(ws.data_ptr()),
                                       ws.numel() * ws.element_size(), _stream_handle(stream)),
           "bf_filter_precomputed")
    return out
