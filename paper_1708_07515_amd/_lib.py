"""ctypes binding of libfdkod.so.  Argument marshalling only.

The library must have been built (``python -m paper_1708_07515_amd.build`` or
``__graft_entry__.build()``); importing the binding without it raises, there
is no fallback path.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

STORE_TYPES = {"f32": 0, "f16": 1, "bf16": 2}
_STORE_BYTES = {0: 4, 1: 2, 2: 2}
NOALLOC_SCRATCH_BYTES = 256 << 20     # FDKOD_NOALLOC_SCRATCH_BYTES of the C header

FDKOD_OK = 0
STATUS_NAMES = {0: "OK", 1: "E_ARG", 2: "E_GEOMETRY", 3: "E_UNSUPPORTED", 4: "E_NOMEM",
                5: "E_HIP", 6: "E_STATE"}


class FdkodError(RuntimeError):
    def __init__(self, status, text):
        self.status = status
        self.code = STATUS_NAMES.get(status, str(status))
        super().__init__(f"fdkod {self.code}: {text}")


class Params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nz", ctypes.c_int32), ("p", ctypes.c_int32),
                ("r", ctypes.c_double), ("s", ctypes.c_int32), ("skip", ctypes.c_int32),
                ("store", ctypes.c_int32), ("decim", ctypes.c_int32), ("taps", ctypes.c_int32),
                ("rows", ctypes.c_int32), ("interp", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("squares", ctypes.c_int32), ("p_dec", ctypes.c_int32), ("d", ctypes.c_int32),
                ("fft_len", ctypes.c_int32), ("max_width", ctypes.c_int32),
                ("z_run", ctypes.c_int32), ("filtered_bytes", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_int64), ("volume_bytes", ctypes.c_int64),
                ("updates", ctypes.c_int64)]


class Tuning(ctypes.Structure):
    _fields_ = [("z_run", ctypes.c_int32), ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("angles_per_stage", ctypes.c_int32), ("decim_chunks", ctypes.c_int32),
                ("bp_ms", ctypes.c_float), ("decim_ms", ctypes.c_float)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_VP = ctypes.c_void_p
EXPORTS = {
    "fdkod_validate": (ctypes.c_int, [ctypes.POINTER(Params)]),
    "fdkod_plan_create": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "fdkod_plan_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "fdkod_plan_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Info)]),
    "fdkod_bounds": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "fdkod_filter": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p]),
    "fdkod_decompose": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "fdkod_reconstruct": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]),
    "fdkod_backproject": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p]),
    "fdkod_get_bounds": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 7),
    "fdkod_backproject_noalloc": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "fdkod_check_counts": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int64), ctypes.c_int32, ctypes.c_int32]),
    "fdkod_cost_counts": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_int64)]),
    "fdkod_choose_s": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                      ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]),
    "fdkod_get_tuning": (ctypes.c_int, [_VP, ctypes.POINTER(Tuning)]),
    "fdkod_set_tuning": (ctypes.c_int, [_VP, ctypes.POINTER(Tuning)]),
    "fdkod_tune": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, ctypes.POINTER(Tuning)]),
    "fdkod_batch_create": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_int32, ctypes.c_int,
                                          ctypes.POINTER(_VP)]),
    "fdkod_batch_destroy": (ctypes.c_int, [_VP]),
    "fdkod_batch_plan": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.POINTER(_VP)]),
    "fdkod_batch_bind": (ctypes.c_int, [_VP, ctypes.POINTER(_VP), ctypes.POINTER(_VP),
                                        ctypes.POINTER(_VP), ctypes.POINTER(_VP)]),
    "fdkod_batch_run": (ctypes.c_int, [_VP, _VP]),
    "fdkod_batch_capture": (ctypes.c_int, [_VP, _VP]),
    "fdkod_batch_replay": (ctypes.c_int, [_VP, _VP]),
    "fdkod_batch_tune": (ctypes.c_int, [_VP, _VP, ctypes.POINTER(Tuning)]),
    "fdkod_batch_info": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)]),
    "fdkod_learned_decompose": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "fdkod_learned_backward": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP]),
    "fdkod_reconstruct_adjoint": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "fdkod_learned_decompose_band": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, ctypes.c_int32, _VP, _VP, _VP]),
    "fdkod_learned_backward_band": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, ctypes.c_int32, _VP, _VP, _VP,
                                                   _VP]),
    "fdkod_reconstruct_adjoint_slab": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                      ctypes.c_int32, _VP, _VP]),
    "fdkod_sq_residual": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_int64, _VP]),
    "fdkod_sq_residual_weighted": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_int64, ctypes.c_float, _VP]),
    "fdkod_adamw_step": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, ctypes.c_int32, ctypes.c_int32]
                         + [ctypes.c_float] * 5 + [_VP]),
    "fdkod_band_rows": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32)]),
    "fdkod_filter_band": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, ctypes.c_int32, _VP, _VP]),
    "fdkod_decompose_band": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, ctypes.c_int32, _VP, _VP]),
    "fdkod_reconstruct_slab": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_int32, _VP, _VP]),
    "fdkod_streamed_bytes": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]),
    "fdkod_reconstruct_streamed": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int32, _VP, ctypes.c_int64, _VP, _VP]),
    "fdkod_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "fdkod_last_error": (ctypes.c_char_p, []),
    "fdkod_version": (ctypes.c_int32, []),
}


def library_path():
    return os.environ.get("FDKOD_LIB", os.path.join(HERE, "libfdkod.so"))


def load_library():
    """Load libfdkod.so and declare its signatures.  Raises if it is missing."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with python -m paper_1708_07515_amd.build")
    lib = ctypes.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def _check(status):
    if status != FDKOD_OK:
        lib = load_library()
        raise FdkodError(status, lib.fdkod_last_error().decode())


DECIM_TYPES = {"triangle": 0, "sinc": 1}      # window of the angular decimation
ROWS_TYPES = {"detector": 0, "cone": 1}       # plain or cone-corrected rows
INTERP_TYPES = {"linear": 0, "cubic": 1}      # interpolation of the crop's shift


def _enum(value, table):
    return table[value] if isinstance(value, str) else int(value)


def _params(n, p, r, s=0, skip=0, nz=0, store="f32", decim="triangle", taps=0, rows="detector",
            interp="linear"):
    return Params(int(n), int(nz), int(p), float(r), int(s), int(skip), _enum(store, STORE_TYPES),
                  _enum(decim, DECIM_TYPES), int(taps), _enum(rows, ROWS_TYPES), _enum(interp, INTERP_TYPES))


def validate(n, p, r, s=0, skip=0, nz=0, store="f32", decim="triangle", taps=0, rows="detector",
             interp="linear"):
    """Host-only parameter check (no device needed)."""
    prm = _params(n, p, r, s, skip, nz, store, decim, taps, rows, interp)
    _check(load_library().fdkod_validate(ctypes.byref(prm)))


LEARNED_PARAMS = 817


# Cost constants of the FP32 kernels on one MI355X, ms per voxel-angle update
# of the reconstruction and per cropped sample of the decomposition (fitted
# by study.py's time split; see cost_counts and choose_s).
MI355X_COSTS = (3.7e-10, 3.7e-10)


def cost_counts(n, p, r, s=0, skip=0, nz=0, **kw):
    """(cropped samples, voxel-angle updates) of one reconstruction, the two
    counts of the cost model (eq. (6)-(7))."""
    lib = load_library()
    prm = _params(n, p, r, s, skip, nz, **kw)
    cropped, updates = ctypes.c_int64(), ctypes.c_int64()
    _check(lib.fdkod_cost_counts(ctypes.byref(prm), ctypes.byref(cropped), ctypes.byref(updates)))
    return cropped.value, updates.value


def choose_s(n, p, r, skip=0, nz=0, s_max=6, costs=MI355X_COSTS, **kw):
    """The s with the least predicted time (eq. (8) over the exact counts)
    and that time in ms."""
    lib = load_library()
    prm = _params(n, p, r, 0, 0, nz, **kw)
    prm.skip = int(skip)
    s_out, ms = ctypes.c_int32(), ctypes.c_double()
    _check(lib.fdkod_choose_s(ctypes.byref(prm), int(s_max), float(costs[0]), float(costs[1]),
                              ctypes.byref(s_out), ctypes.byref(ms)))
    return s_out.value, ms.value


def check_counts(reset=True):
    """Event counts of a checked build (list of 4 ints, see fdkod.h); raises
    E_UNSUPPORTED on an unchecked build."""
    lib = load_library()
    arr = (ctypes.c_int64 * 4)()
    _check(lib.fdkod_check_counts(arr, 4, 1 if reset else 0))
    return [int(x) for x in arr]


def _dev_tensor(t, dtype, name, numel=None):
    if t is None or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must hold {numel} elements")


def sq_residual(f, ref, resid, loss, stream=None):
    """resid = 2 (f - ref), loss[0] = sum (f - ref)^2 (float64 device scalar)."""
    import torch
    for t, nm in ((f, "f"), (ref, "ref"), (resid, "resid")):
        _dev_tensor(t, torch.float32, nm, f.numel())
    _dev_tensor(loss, torch.float64, "loss", 1)
    _check(load_library().fdkod_sq_residual(
        ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(ref.data_ptr()),
        ctypes.c_void_p(resid.data_ptr()), ctypes.c_void_p(loss.data_ptr()), f.numel(),
        _stream_ptr(stream)))


def sq_residual_weighted(f, ref, resid, loss, weight, stream=None):
    """resid = 2 w (f - ref), loss[0] = w sum (f - ref)^2."""
    import torch
    for t, nm in ((f, "f"), (ref, "ref"), (resid, "resid")):
        _dev_tensor(t, torch.float32, nm, f.numel())
    _dev_tensor(loss, torch.float64, "loss", 1)
    _check(load_library().fdkod_sq_residual_weighted(
        ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(ref.data_ptr()),
        ctypes.c_void_p(resid.data_ptr()), ctypes.c_void_p(loss.data_ptr()), f.numel(), float(weight),
        _stream_ptr(stream)))


def adamw_step(master, m1, m2, grad, w_bf16, step, lr, beta1=0.9, beta2=0.999, eps=1e-8,
               weight_decay=0.0, stream=None):
    """One AdamW step on the device; refreshes the BF16 copy w_bf16."""
    import torch
    n = master.numel()
    for t, nm in ((master, "master"), (m1, "m1"), (m2, "m2"), (grad, "grad")):
        _dev_tensor(t, torch.float32, nm, n)
    _dev_tensor(w_bf16, torch.bfloat16, "w_bf16", n)
    _check(load_library().fdkod_adamw_step(
        *(ctypes.c_void_p(t.data_ptr()) for t in (master, m1, m2, grad, w_bf16)), n, int(step),
        float(lr), float(beta1), float(beta2), float(eps), float(weight_decay), _stream_ptr(stream)))


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """An FDK-OD plan: geometry tables on one device, sizes of the buffers."""

    def __init__(self, n, p, r, s=0, skip=0, nz=0, store="f32", device=0, decim="triangle", taps=0,
                 rows="detector", interp="linear", _handle=None):
        """decim: "triangle" or "sinc" (taps 2, 4 or 6; 0 = 4); rows: "detector"
        or "cone" (cone-corrected); interp: "linear" or "cubic" shift."""
        self._lib = load_library()
        self.params = _params(n, p, r, s, skip, nz, store, decim, taps, rows, interp)
        self.decim, self.taps = self.params.decim, self.params.taps
        self.rows, self.interp = self.params.rows, self.params.interp
        self.n, self.p, self.r, self.s, self.skip = int(n), int(p), float(r), int(s), int(skip)
        self.nz = int(nz) or int(n)
        self.store = self.params.store
        self.device = int(device)
        self._owned = _handle is None
        if _handle is None:
            h = ctypes.c_void_p()
            _check(self._lib.fdkod_plan_create(ctypes.byref(self.params), self.device, ctypes.byref(h)))
        else:
            h = _handle
        self._h = h
        info = Info()
        _check(self._lib.fdkod_plan_info(h, ctypes.byref(info)))
        self.info = info

    # kernel shapes ----------------------------------------------------------
    def get_tuning(self):
        t = Tuning()
        _check(self._lib.fdkod_get_tuning(self._h, ctypes.byref(t)))
        return t.as_dict()

    def set_tuning(self, **kw):
        t = Tuning()
        _check(self._lib.fdkod_get_tuning(self._h, ctypes.byref(t)))
        for k, v in kw.items():
            setattr(t, k, v)
        _check(self._lib.fdkod_set_tuning(self._h, ctypes.byref(t)))

    def tune(self, filt, ws, vol, stream=None):
        """Autotune on the given buffers (overwrites vol and ws); returns the choice."""
        t = Tuning()
        _check(self._lib.fdkod_tune(self._h, ctypes.c_void_p(filt.data_ptr()),
                                    ctypes.c_void_p(ws.data_ptr() if ws is not None else 0),
                                    ctypes.c_void_p(vol.data_ptr()), _stream_ptr(stream),
                                    ctypes.byref(t)))
        return t.as_dict()

    # sizes ---------------------------------------------------------------
    @property
    def p_dec(self):
        return self.info.p_dec

    @property
    def squares(self):
        return self.info.squares

    @property
    def workspace_bytes(self):
        return self.info.workspace_bytes

    @property
    def filtered_bytes(self):
        return self.info.filtered_bytes

    @property
    def updates(self):
        return self.info.updates

    def store_torch_dtype(self):
        import torch
        return {0: torch.float32, 1: torch.float16, 2: torch.bfloat16}[self.store]

    # buffer helpers (allocation happens here, in torch, never in the library)
    def empty_filtered(self):
        import torch
        return torch.empty((self.p, self.n, self.n), dtype=self.store_torch_dtype(),
                           device=f"cuda:{self.device}")

    def empty_workspace(self):
        import torch
        nbytes = max(int(self.workspace_bytes), 256)
        return torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{self.device}")

    def empty_volume(self):
        import torch
        return torch.empty((self.nz, self.n, self.n), dtype=torch.float32,
                           device=f"cuda:{self.device}")

    # checks ----------------------------------------------------------------
    def _chk(self, t, shape, dtype, name):
        if t is None:
            raise ValueError(f"{name} is None")
        if not t.is_cuda or t.device.index != self.device:
            raise ValueError(f"{name} must live on cuda:{self.device}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
        if t.dtype != dtype:
            raise ValueError(f"{name} has dtype {t.dtype}, expected {dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")

    def _chk_ws(self, ws):
        if self.s == 0:
            return
        if ws is None or not ws.is_cuda or ws.numel() * ws.element_size() < self.workspace_bytes:
            raise ValueError(f"workspace must hold {self.workspace_bytes} bytes on the device")
        if not ws.is_contiguous():
            raise ValueError("workspace must be contiguous")

    # enqueueing calls ----------------------------------------------------
    def bounds(self, stream=None):
        _check(self._lib.fdkod_bounds(self._h, _stream_ptr(stream)))

    def filter(self, proj, filt, stream=None):
        import torch
        self._chk(proj, (self.p, self.n, self.n), torch.float32, "proj")
        self._chk(filt, (self.p, self.n, self.n), self.store_torch_dtype(), "filt")
        _check(self._lib.fdkod_filter(self._h, ctypes.c_void_p(proj.data_ptr()),
                                      ctypes.c_void_p(filt.data_ptr()), _stream_ptr(stream)))

    def decompose(self, filt, ws, stream=None):
        self._chk(filt, (self.p, self.n, self.n), self.store_torch_dtype(), "filt")
        self._chk_ws(ws)
        _check(self._lib.fdkod_decompose(self._h, ctypes.c_void_p(filt.data_ptr()),
                                         ctypes.c_void_p(ws.data_ptr() if ws is not None else 0),
                                         _stream_ptr(stream)))

    def reconstruct(self, filt, ws, vol, stream=None):
        import torch
        self._chk(vol, (self.nz, self.n, self.n), torch.float32, "vol")
        if self.s == 0:
            self._chk(filt, (self.p, self.n, self.n), self.store_torch_dtype(), "filt")
        else:
            self._chk_ws(ws)
        _check(self._lib.fdkod_reconstruct(
            self._h, ctypes.c_void_p(filt.data_ptr() if filt is not None else 0),
            ctypes.c_void_p(ws.data_ptr() if ws is not None else 0),
            ctypes.c_void_p(vol.data_ptr()), _stream_ptr(stream)))

    def backproject(self, filt, vol, ws=None, stream=None):
        import torch
        self._chk(filt, (self.p, self.n, self.n), self.store_torch_dtype(), "filt")
        self._chk(vol, (self.nz, self.n, self.n), torch.float32, "vol")
        self._chk_ws(ws)
        _check(self._lib.fdkod_backproject(
            self._h, ctypes.c_void_p(filt.data_ptr()), ctypes.c_void_p(vol.data_ptr()),
            ctypes.c_void_p(ws.data_ptr() if ws is not None else 0), _stream_ptr(stream)))

    def backproject_noalloc(self, filt, vol, stream=None):
        """fdkod_backproject with the library's fixed device array as the
        workspace (nothing is allocated; plans whose workspace exceeds
        NOALLOC_SCRATCH_BYTES raise E_UNSUPPORTED)."""
        import torch
        self._chk(filt, (self.p, self.n, self.n), self.store_torch_dtype(), "filt")
        self._chk(vol, (self.nz, self.n, self.n), torch.float32, "vol")
        _check(self._lib.fdkod_backproject_noalloc(
            self._h, ctypes.c_void_p(filt.data_ptr()), ctypes.c_void_p(vol.data_ptr()), _stream_ptr(stream)))

    # learned decimation ---------------------------------------------------
    @property
    def workspace_elems(self):
        return int(self.workspace_bytes) // _STORE_BYTES[self.store]

    def _chk_weights(self, w):
        import torch
        self._chk(w, (LEARNED_PARAMS,), torch.bfloat16, "weights")

    def _chk_dws(self, dws):
        import torch
        self._chk(dws, (self.workspace_elems,), torch.float32, "dws")

    def learned_decompose(self, filt, ws, weights, stream=None):
        """Triangle decimation plus the learned correction (ws receives Y)."""
        self._chk(filt, (self.p, self.n, self.n), self.store_torch_dtype(), "filt")
        self._chk_ws(ws)
        self._chk_weights(weights)
        _check(self._lib.fdkod_learned_decompose(
            self._h, ctypes.c_void_p(filt.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
            ctypes.c_void_p(weights.data_ptr()), _stream_ptr(stream)))

    def learned_backward(self, filt, dws, weights, grad, stream=None):
        """grad = d/dweights of sum(R * dws) (float32 [817], overwritten)."""
        import torch
        self._chk(filt, (self.p, self.n, self.n), self.store_torch_dtype(), "filt")
        self._chk_dws(dws)
        self._chk_weights(weights)
        self._chk(grad, (LEARNED_PARAMS,), torch.float32, "grad")
        _check(self._lib.fdkod_learned_backward(
            self._h, ctypes.c_void_p(filt.data_ptr()), ctypes.c_void_p(dws.data_ptr()),
            ctypes.c_void_p(weights.data_ptr()), ctypes.c_void_p(grad.data_ptr()),
            _stream_ptr(stream)))

    def reconstruct_adjoint(self, resid, dws, stream=None):
        """dws = transpose of the reconstruction applied to resid."""
        import torch
        self._chk(resid, (self.nz, self.n, self.n), torch.float32, "resid")
        self._chk_dws(dws)
        _check(self._lib.fdkod_reconstruct_adjoint(
            self._h, ctypes.c_void_p(resid.data_ptr()), ctypes.c_void_p(dws.data_ptr()),
            _stream_ptr(stream)))

    # low-memory slabs -----------------------------------------------------
    def band_rows(self, z0, nzs):
        """Detector rows (v0, nrows) that slices [z0, z0 + nzs) sample."""
        v0, nr = ctypes.c_int32(), ctypes.c_int32()
        _check(self._lib.fdkod_band_rows(self._h, int(z0), int(nzs), ctypes.byref(v0), ctypes.byref(nr)))
        return v0.value, nr.value

    def band_workspace_elems(self, nrows):
        return (int(self.workspace_bytes) // _STORE_BYTES[self.store]) // self.n * int(nrows)

    def empty_band(self, nrows):
        """(projection band, filtered band, workspace band) for nrows rows."""
        import torch
        dev = f"cuda:{self.device}"
        proj = torch.empty((self.p, nrows, self.n), dtype=torch.float32, device=dev)
        filt = torch.empty((self.p, nrows, self.n), dtype=self.store_torch_dtype(), device=dev)
        ws = torch.empty(max(self.band_workspace_elems(nrows), 1), dtype=self.store_torch_dtype(), device=dev)
        return proj, filt, ws

    def filter_band(self, proj_band, v0, filt_band, stream=None):
        import torch
        nr = proj_band.shape[1]
        self._chk(proj_band, (self.p, nr, self.n), torch.float32, "proj_band")
        self._chk(filt_band, (self.p, nr, self.n), self.store_torch_dtype(), "filt_band")
        _check(self._lib.fdkod_filter_band(self._h, ctypes.c_void_p(proj_band.data_ptr()), int(v0), nr,
                                           ctypes.c_void_p(filt_band.data_ptr()), _stream_ptr(stream)))

    def decompose_band(self, filt_band, v0, ws_band, stream=None):
        nr = filt_band.shape[1]
        self._chk(filt_band, (self.p, nr, self.n), self.store_torch_dtype(), "filt_band")
        if self.s > 0 and (ws_band is None or ws_band.numel() < self.band_workspace_elems(nr)):
            raise ValueError("workspace band too small")
        _check(self._lib.fdkod_decompose_band(
            self._h, ctypes.c_void_p(filt_band.data_ptr()), int(v0), nr,
            ctypes.c_void_p(ws_band.data_ptr() if ws_band is not None else 0), _stream_ptr(stream)))

    def reconstruct_slab(self, filt_band, ws_band, v0, nrows, z0, vol_slab, stream=None):
        import torch
        nzs = vol_slab.shape[0]
        self._chk(vol_slab, (nzs, self.n, self.n), torch.float32, "vol_slab")
        _check(self._lib.fdkod_reconstruct_slab(
            self._h, ctypes.c_void_p(filt_band.data_ptr() if filt_band is not None else 0),
            ctypes.c_void_p(ws_band.data_ptr() if ws_band is not None else 0), int(v0), int(nrows), int(z0),
            nzs, ctypes.c_void_p(vol_slab.data_ptr()), _stream_ptr(stream)))

    # the learned filter on bands (training on slabs) ---------------------
    def learned_decompose_band(self, filt_band, v0, ws_band, weights, stream=None):
        nr = filt_band.shape[1]
        self._chk(filt_band, (self.p, nr, self.n), self.store_torch_dtype(), "filt_band")
        if ws_band.numel() * ws_band.element_size() < self.band_workspace_elems(nr) * _STORE_BYTES[self.store]:
            raise ValueError("workspace band too small")
        self._chk_weights(weights)
        _check(self._lib.fdkod_learned_decompose_band(
            self._h, ctypes.c_void_p(filt_band.data_ptr()), int(v0), nr, ctypes.c_void_p(ws_band.data_ptr()),
            ctypes.c_void_p(weights.data_ptr()), _stream_ptr(stream)))

    def learned_backward_band(self, filt_band, v0, dws_band, weights, grad, stream=None):
        import torch
        nr = filt_band.shape[1]
        self._chk(filt_band, (self.p, nr, self.n), self.store_torch_dtype(), "filt_band")
        self._chk(dws_band, (self.band_workspace_elems(nr),), torch.float32, "dws_band")
        self._chk_weights(weights)
        self._chk(grad, (LEARNED_PARAMS,), torch.float32, "grad")
        _check(self._lib.fdkod_learned_backward_band(
            self._h, ctypes.c_void_p(filt_band.data_ptr()), int(v0), nr, ctypes.c_void_p(dws_band.data_ptr()),
            ctypes.c_void_p(weights.data_ptr()), ctypes.c_void_p(grad.data_ptr()), _stream_ptr(stream)))

    def reconstruct_adjoint_slab(self, resid_slab, v0, nrows, z0, dws_band, stream=None):
        import torch
        nzs = resid_slab.shape[0]
        self._chk(resid_slab, (nzs, self.n, self.n), torch.float32, "resid_slab")
        self._chk(dws_band, (self.band_workspace_elems(nrows),), torch.float32, "dws_band")
        _check(self._lib.fdkod_reconstruct_adjoint_slab(
            self._h, ctypes.c_void_p(resid_slab.data_ptr()), int(v0), int(nrows), int(z0), nzs,
            ctypes.c_void_p(dws_band.data_ptr()), _stream_ptr(stream)))

    def streamed_bytes(self, nzs):
        b = ctypes.c_int64()
        _check(self._lib.fdkod_streamed_bytes(self._h, int(nzs), ctypes.byref(b)))
        return b.value

    def reconstruct_streamed(self, host_proj, host_vol, nzs, work, stream=None, copy_stream=None):
        """Whole reconstruction from host tensors, slab by slab (synchronous)."""
        import torch
        for t, shape, nm in ((host_proj, (self.p, self.n, self.n), "host_proj"),
                             (host_vol, (self.nz, self.n, self.n), "host_vol")):
            if t.is_cuda or tuple(t.shape) != shape or t.dtype != torch.float32 or not t.is_contiguous():
                raise ValueError(f"{nm} must be a contiguous float32 host tensor of shape {shape}")
        if not work.is_cuda or not work.is_contiguous():
            raise ValueError("work must be a contiguous device tensor")
        _check(self._lib.fdkod_reconstruct_streamed(
            self._h, ctypes.c_void_p(host_proj.data_ptr()), ctypes.c_void_p(host_vol.data_ptr()), int(nzs),
            ctypes.c_void_p(work.data_ptr()), work.numel() * work.element_size(), _stream_ptr(stream),
            _stream_ptr(copy_stream)))

    def get_bounds(self):
        """Bounds tables as numpy arrays (synchronises)."""
        import numpy as np
        nsq, p, pd = self.squares, self.p, self.p_dec
        ac_p = np.zeros((nsq, p), np.float32)
        ac_m = np.zeros((nsq, pd), np.float32)
        amin = np.zeros((nsq, pd), np.float32)
        amax = np.zeros((nsq, pd), np.float32)
        u0 = np.zeros(nsq, np.int32)
        width = np.zeros(nsq, np.int32)
        rect = np.zeros((nsq, 4), np.int32)
        ptr = lambda a: ctypes.c_void_p(a.ctypes.data)  # noqa: E731
        _check(self._lib.fdkod_get_bounds(self._h, ptr(ac_p), ptr(ac_m), ptr(amin), ptr(amax),
                                          ptr(u0), ptr(width), ptr(rect)))
        return dict(ac_p=ac_p, ac_m=ac_m, amin=amin, amax=amax, u0=u0, width=width, rect=rect)

    def close(self):
        if getattr(self, "_h", None) and getattr(self, "_owned", True):
            self._lib.fdkod_plan_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """Many volumes reconstructed together: grouped decimation, one persistent
    backprojection launch, optional hipGraph capture."""

    def __init__(self, volumes, store="f32", device=0):
        """volumes: list of dicts with keys n, p, r and optional s, skip, nz."""
        self._lib = load_library()
        self.device = int(device)
        prms = [_params(v["n"], v["p"], v["r"], v.get("s", 0), v.get("skip", 0), v.get("nz", 0), store,
                        v.get("decim", "triangle"), v.get("taps", 0), v.get("rows", "detector"),
                        v.get("interp", "linear"))
                for v in volumes]
        arr = (Params * len(prms))(*prms)
        h = ctypes.c_void_p()
        _check(self._lib.fdkod_batch_create(arr, len(prms), self.device, ctypes.byref(h)))
        self._h = h
        self.plans = []
        for i, v in enumerate(volumes):
            ph = ctypes.c_void_p()
            _check(self._lib.fdkod_batch_plan(h, i, ctypes.byref(ph)))
            self.plans.append(Plan(v["n"], v["p"], v["r"], v.get("s", 0), v.get("skip", 0),
                                   v.get("nz", 0), store, device, _handle=ph))
        self._bound = None

    def __len__(self):
        return len(self.plans)

    def bind(self, proj, filt, ws, vol):
        """Lists of tensors, one per volume (ws entries may be None for s = 0)."""
        n = len(self.plans)
        for i, pl in enumerate(self.plans):
            import torch
            pl._chk(proj[i], (pl.p, pl.n, pl.n), torch.float32, f"proj[{i}]")
            pl._chk(filt[i], (pl.p, pl.n, pl.n), pl.store_torch_dtype(), f"filt[{i}]")
            pl._chk(vol[i], (pl.nz, pl.n, pl.n), torch.float32, f"vol[{i}]")
            pl._chk_ws(ws[i])
        ptrs = lambda ts: (_VP * n)(*[t.data_ptr() if t is not None else 0 for t in ts])  # noqa: E731
        _check(self._lib.fdkod_batch_bind(self._h, ptrs(proj), ptrs(filt), ptrs(ws), ptrs(vol)))
        self._bound = (list(proj), list(filt), list(ws), list(vol))   # keep the tensors alive

    def run(self, stream=None):
        _check(self._lib.fdkod_batch_run(self._h, _stream_ptr(stream)))

    def capture(self, stream):
        _check(self._lib.fdkod_batch_capture(self._h, ctypes.c_void_p(stream.cuda_stream)))

    def replay(self, stream=None):
        _check(self._lib.fdkod_batch_replay(self._h, _stream_ptr(stream)))

    def tune(self, stream=None):
        t = Tuning()
        _check(self._lib.fdkod_batch_tune(self._h, _stream_ptr(stream), ctypes.byref(t)))
        return t.as_dict()

    def info(self):
        items, blocks, upd = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
        _check(self._lib.fdkod_batch_info(self._h, ctypes.byref(items), ctypes.byref(blocks),
                                          ctypes.byref(upd)))
        return dict(items=items.value, blocks=blocks.value, updates_eq=upd.value)

    def close(self):
        for p in self.plans:
            p._h = None
        if getattr(self, "_h", None):
            self._lib.fdkod_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
