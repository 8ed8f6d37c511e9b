"""ctypes binding of liblbm.so (declared in include/lbm.h).

Argument marshalling only: every step of the update runs in the HIP
library. PyTorch supplies device memory (the context workspace) and the
stream. If the built library is missing this module raises at import
time; there is no fallback path.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

NQ = 41
F64, F32, F16_SHIFT, BF16_SHIFT, F32_SHIFT = 0, 1, 2, 3, 4
FLAG_STOCHASTIC_ROUNDING = 1
FLAG_ISOTHERMAL = 2
FLAG_SERIES_EQUILIBRIUM = 4
FLAG_ENTROPIC = 8
FLAG_WALLS = 16
TAU_LB, TAU_PAPER = 0, 1
SHIFT_AUTO = -1000
STORAGE = {"f64": F64, "f32": F32, "f16s": F16_SHIFT, "bf16s": BF16_SHIFT, "f32s": F32_SHIFT}
ELEM_BYTES = {"f64": 8, "f32": 4, "f16s": 2, "bf16s": 2, "f32s": 4}

OK, E_ARG, E_NOMEM, E_DOMAIN, E_NONFINITE, E_HIP, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6


class LbmError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__("%s: %s (%d)" % (what, lib().lbm_strerror(code).decode(), code))


class Box(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("tau", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("storage", ctypes.c_int32), ("tau_conv", ctypes.c_int32), ("rho0", ctypes.c_double),
                ("newton_iters", ctypes.c_int32), ("shift_exp", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("seed", ctypes.c_uint32)]


class Info(ctypes.Structure):
    _fields_ = [("storage", ctypes.c_int32), ("newton_iters", ctypes.c_int32), ("shift_exp", ctypes.c_int32),
                ("nboxes", ctypes.c_int32), ("nodes", ctypes.c_int64), ("bytes_per_step", ctypes.c_int64),
                ("block_threads", ctypes.c_int32), ("variant", ctypes.c_int32), ("device_bytes", ctypes.c_uint64),
                ("flags", ctypes.c_uint32), ("steps_done", ctypes.c_uint32)]


class Tuning(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("xcd_remap", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("graph_steps", ctypes.c_int32)]


# lbm_schedule: one launch per box, or one launch over every (box, tile)
class TuneResult(ctypes.Structure):
    _fields_ = [("best", Tuning), ("best_ms", ctypes.c_float), ("from_cache", ctypes.c_int32),
                ("timed", ctypes.c_int32)]


SCHEDULES = {"per_box": 0, "batched": 1}
TUNE_SCHEDULE, TUNE_GRAPH, TUNE_CACHE = 1, 2, 4
GRAPH_STEPS_MAX = 1024


_dp = ctypes.POINTER(ctypes.c_double)
_lp = ctypes.POINTER(ctypes.c_int64)
_vp = ctypes.c_void_p

# every symbol of include/lbm.h with its C signature
SIGNATURES = {
    "lbm_lattice": (ctypes.c_int, [_dp, _dp, _dp]),
    "lbm_workspace_size": (ctypes.c_int, [ctypes.POINTER(Box), ctypes.c_int32, ctypes.POINTER(Opts),
                                          ctypes.POINTER(ctypes.c_uint64)]),
    "lbm_init": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.POINTER(Box), ctypes.c_int32, ctypes.POINTER(Opts),
                                _dp, _dp, _dp, _dp, _dp, _vp, _vp, ctypes.c_uint64]),
    "lbm_init_device": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.POINTER(Box), ctypes.c_int32, ctypes.POINTER(Opts),
                                       _vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_uint64]),
    "lbm_step": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "lbm_synchronize": (ctypes.c_int, [_vp]),
    "lbm_moments": (ctypes.c_int, [_vp, _dp, _dp, _dp, _dp, _dp]),
    "lbm_totals": (ctypes.c_int, [_vp, _dp]),
    "lbm_status": (ctypes.c_int, [_vp]),
    "lbm_project": (ctypes.c_int, [_vp, ctypes.c_int32, _dp, _dp]),
    "lbm_get_populations": (ctypes.c_int, [_vp, _dp]),
    "lbm_set_populations": (ctypes.c_int, [_vp, _dp]),
    "lbm_gather": (ctypes.c_int, [_vp, ctypes.c_int32, _lp, ctypes.c_int64, _dp]),
    "lbm_debug_pull_map": (ctypes.c_int, [_vp, ctypes.c_int32, _lp]),
    "lbm_get_info": (ctypes.c_int, [_vp, ctypes.POINTER(Info)]),
    "lbm_set_step_counter": (ctypes.c_int, [_vp, ctypes.c_uint32]),
    "lbm_set_walls": (ctypes.c_int, [_vp, ctypes.c_int32, _dp]),
    "lbm_set_walls_kind": (ctypes.c_int, [_vp, ctypes.c_int32, _dp, ctypes.POINTER(ctypes.c_int32)]),
    "lbm_num_variants": (ctypes.c_int, []),
    "lbm_variant_desc": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_uint32)]),
    "lbm_set_tuning": (ctypes.c_int, [_vp, ctypes.POINTER(Tuning)]),
    "lbm_get_tuning": (ctypes.c_int, [_vp, ctypes.POINTER(Tuning)]),
    "lbm_autotune": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(Tuning)]),
    "lbm_autotune_ex": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_uint32, ctypes.POINTER(ctypes.c_float),
                                       ctypes.POINTER(TuneResult)]),
    "lbm_stream_free": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "lbm_device_copy": (ctypes.c_int, [_vp, _vp, ctypes.c_uint64, _vp]),
    "lbm_totals_noalloc": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(Box), ctypes.c_uint64, ctypes.c_double,
                                          ctypes.c_int32, _vp, _vp]),
    "lbm_tune_cache_file": (ctypes.c_int, [ctypes.c_char_p]),
    "lbm_tune_cache_clear": (ctypes.c_int, []),
    "lbm_tune_cache_count": (ctypes.c_int, []),
    "lbm_stream": (_vp, [_vp]),
    "lbm_free": (None, [_vp]),
    "lbm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "lbm_selftest": (ctypes.c_int, []),
    "lbm_collide_host": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32, ctypes.c_double, _dp, _dp]),
}

_lib = None


def lib():
    """The loaded liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("liblbm.so is not built (run __graft_entry__.build()); "
                              "the GPU path has no fallback")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc, what):
    if rc != OK:
        raise LbmError(rc, what)


def _d(a):
    return a.ctypes.data_as(_dp)


def lattice():
    """(c[41,3], w[41], theta0) as the library holds them."""
    c = np.zeros((NQ, 3))
    w = np.zeros(NQ)
    t = np.zeros(1)
    _check(lib().lbm_lattice(_d(c), _d(w), _d(t)), "lbm_lattice")
    return c, w, float(t[0])


def _boxes(boxes):
    arr = (Box * len(boxes))()
    for i, b in enumerate(boxes):
        nx, ny, nz, tau = b
        arr[i] = Box(int(nx), int(ny), int(nz), 0, float(tau))
    return arr


def _opts(storage, tau_conv, rho0, newton_iters, shift_exp, stochastic=False, seed=0, isothermal=False, series=False,
          entropic=False, walls=False):
    st = STORAGE[storage] if isinstance(storage, str) else int(storage)
    flags = ((FLAG_STOCHASTIC_ROUNDING if stochastic else 0) | (FLAG_ISOTHERMAL if isothermal else 0)
             | (FLAG_SERIES_EQUILIBRIUM if series else 0) | (FLAG_ENTROPIC if entropic else 0)
             | (FLAG_WALLS if walls else 0))
    return Opts(st, int(tau_conv), float(rho0), int(newton_iters),
                SHIFT_AUTO if shift_exp is None else int(shift_exp), flags, int(seed) & 0xffffffff)


def workspace_size(boxes, storage="f32", tau_conv=TAU_LB, rho0=1.0, newton_iters=0, shift_exp=None,
                   stochastic=False, isothermal=False, series=False, entropic=False, walls=False):
    bx = _boxes(boxes)
    op = _opts(storage, tau_conv, rho0, newton_iters, shift_exp, stochastic, 0, isothermal, series, entropic, walls)
    out = ctypes.c_uint64(0)
    _check(lib().lbm_workspace_size(bx, len(boxes), ctypes.byref(op), ctypes.byref(out)), "lbm_workspace_size")
    return int(out.value)


class Context:
    """A live lbm_ctx. Methods are the C entry points without the prefix."""

    def __init__(self, handle, boxes, workspace, stream):
        self._h = handle
        self.boxes = [tuple(b) for b in boxes]
        self._workspace = workspace  # keeps the torch allocation alive
        self._stream = stream
        self.box_nodes = [2 * b[0] * b[1] * b[2] for b in self.boxes]
        self.nodes = sum(self.box_nodes)

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("context already freed")
        return self._h

    def step(self, n=1):
        _check(lib().lbm_step(self.handle, int(n)), "lbm_step")

    def stream_free(self, n=1):
        """n collisionless streaming steps (an exact permutation of the held values)."""
        _check(lib().lbm_stream_free(self.handle, int(n)), "lbm_stream_free")

    def synchronize(self):
        _check(lib().lbm_synchronize(self.handle), "lbm_synchronize")

    def moments(self):
        """(5, nodes) array: rho, jx, jy, jz, E per node (FP64)."""
        m = np.zeros((5, self.nodes))
        _check(lib().lbm_moments(self.handle, *[_d(m[k]) for k in range(5)]), "lbm_moments")
        return m

    def totals(self, check=True):
        """(nboxes, 5): mass, Jx, Jy, Jz, E per box, summed in FP64 on the device."""
        out = np.zeros((len(self.boxes), 5))
        rc = lib().lbm_totals(self.handle, _d(out))
        if check:
            _check(rc, "lbm_totals")
        return out

    def status(self):
        return int(lib().lbm_status(self.handle))

    def project(self, box, k):
        """Complex Fourier amplitudes of (rho, jx, jy, jz, E, theta) of one box
        at wavevector k (radians per cell), computed on the device."""
        kv = np.ascontiguousarray(k, dtype=np.float64).reshape(3)
        out = np.zeros(12)
        _check(lib().lbm_project(self.handle, int(box), _d(kv), _d(out)), "lbm_project")
        return out[0::2] + 1j * out[1::2]

    def get_populations(self):
        f = np.zeros(NQ * self.nodes)
        _check(lib().lbm_get_populations(self.handle, _d(f)), "lbm_get_populations")
        return f

    def set_walls(self, box, lower, upper, kinds=("diffuse", "diffuse")):
        """lbm_set_walls_kind: (ux, uy, uz, theta) of the lower and the upper
        wall of one box (theta absolute) and their kinds ("diffuse" or
        "specular")."""
        w = np.ascontiguousarray(list(lower) + list(upper), dtype=np.float64)
        if w.size != 8:
            raise ValueError("two (ux, uy, uz, theta) expected")
        names = {"diffuse": 0, "specular": 1}
        k = (ctypes.c_int32 * 2)(*[names[x] if isinstance(x, str) else int(x) for x in kinds])
        _check(lib().lbm_set_walls_kind(self.handle, int(box), _d(w), k), "lbm_set_walls_kind")

    def set_populations(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        if f.size != NQ * self.nodes:
            raise ValueError("expected %d values" % (NQ * self.nodes))
        _check(lib().lbm_set_populations(self.handle, _d(f)), "lbm_set_populations")

    def gather(self, box, idx):
        idx = np.ascontiguousarray(idx, dtype=np.int64).reshape(-1)
        out = np.zeros(idx.size)
        _check(lib().lbm_gather(self.handle, int(box), idx.ctypes.data_as(_lp), idx.size, _d(out)), "lbm_gather")
        return out

    def debug_pull_map(self, box=0):
        n = self.box_nodes[box]
        out = np.zeros(NQ * n, dtype=np.int64)
        _check(lib().lbm_debug_pull_map(self.handle, int(box), out.ctypes.data_as(_lp)), "lbm_debug_pull_map")
        return out.reshape(NQ, n)

    def set_step_counter(self, n):
        _check(lib().lbm_set_step_counter(self.handle, int(n)), "lbm_set_step_counter")

    def info(self):
        i = Info()
        _check(lib().lbm_get_info(self.handle, ctypes.byref(i)), "lbm_get_info")
        return {k: getattr(i, k) for k, _ in Info._fields_}

    def stream(self):
        return lib().lbm_stream(self.handle)

    def set_tuning(self, variant=None, xcd_remap=None, schedule=None, graph_steps=None):
        """Change any of the launch settings (the others are kept). schedule:
        "per_box" or "batched"; graph_steps: 0 or an even count of steps per
        captured graph."""
        t = Tuning()
        _check(lib().lbm_get_tuning(self.handle, ctypes.byref(t)), "lbm_get_tuning")
        if variant is not None:
            t.variant = int(variant)
        if xcd_remap is not None:
            t.xcd_remap = int(xcd_remap)
        if schedule is not None:
            t.schedule = SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule)
        if graph_steps is not None:
            t.graph_steps = int(graph_steps)
        _check(lib().lbm_set_tuning(self.handle, ctypes.byref(t)), "lbm_set_tuning")

    def get_tuning(self):
        """(variant, xcd_remap) of the step kernel."""
        t = Tuning()
        _check(lib().lbm_get_tuning(self.handle, ctypes.byref(t)), "lbm_get_tuning")
        return t.variant, t.xcd_remap

    def tuning(self):
        """Every launch setting as a dict."""
        t = Tuning()
        _check(lib().lbm_get_tuning(self.handle, ctypes.byref(t)), "lbm_get_tuning")
        names = {v: k for k, v in SCHEDULES.items()}
        return {"variant": t.variant, "xcd_remap": t.xcd_remap, "schedule": names.get(t.schedule, t.schedule),
                "graph_steps": t.graph_steps}

    def autotune(self, reps=3):
        """Times every launch configuration, keeps the fastest; returns
        ((variant, xcd_remap), {(variant, xcd_remap): ms per step})."""
        nv = num_variants()
        ms = (ctypes.c_float * (2 * nv))()
        best = Tuning()
        _check(lib().lbm_autotune(self.handle, int(reps), ms, ctypes.byref(best)), "lbm_autotune")
        return (best.variant, best.xcd_remap), {(v, x): ms[2 * v + x] for v in range(nv) for x in range(2)}

    def autotune_ex(self, reps=3, schedule=True, graph=True, cache=True):
        """The wider search with the tuning cache (lbm_autotune_ex): returns
        a dict with the chosen settings, best_ms, from_cache and timed."""
        flags = (TUNE_SCHEDULE if schedule else 0) | (TUNE_GRAPH if graph else 0) | (TUNE_CACHE if cache else 0)
        r = TuneResult()
        _check(lib().lbm_autotune_ex(self.handle, int(reps), flags, None, ctypes.byref(r)), "lbm_autotune_ex")
        names = {v: k for k, v in SCHEDULES.items()}
        return {"variant": r.best.variant, "xcd_remap": r.best.xcd_remap,
                "schedule": names.get(r.best.schedule, r.best.schedule), "graph_steps": r.best.graph_steps,
                "best_ms": r.best_ms, "from_cache": bool(r.from_cache), "timed": r.timed}

    def free(self):
        if self._h is not None:
            lib().lbm_free(self._h)
            self._h = None
            self._workspace = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def init(boxes, rho, ux, uy, uz, theta, storage="f32", tau_conv=TAU_LB, rho0=1.0, newton_iters=0,
         shift_exp=None, stream=None, torch_workspace=True, stochastic=False, seed=0, isothermal=False,
         series=False, entropic=False, walls=False):
    """lbm_init. boxes: [(nx, ny, nz, tau), ...]; nodal FP64 fields of all
    boxes concatenated (theta absolute; not used by the isothermal model).
    stream: a torch.cuda.Stream (or None for the library's own). With
    torch_workspace the device memory is a torch uint8 tensor held by the
    returned Context."""
    bx = _boxes(boxes)
    op = _opts(storage, tau_conv, rho0, newton_iters, shift_exp, stochastic, seed, isothermal, series, entropic,
               walls)
    arrs = [np.ascontiguousarray(a, dtype=np.float64).reshape(-1) for a in (rho, ux, uy, uz, theta)]
    nodes = sum(2 * b[0] * b[1] * b[2] for b in boxes)
    for a in arrs:
        if a.size != nodes:
            raise ValueError("field has %d values, boxes have %d nodes" % (a.size, nodes))
    ws = None
    ws_ptr, ws_bytes = None, 0
    if torch_workspace:
        import torch
        ws_bytes = workspace_size(boxes, storage, tau_conv, rho0, newton_iters, shift_exp, stochastic, isothermal,
                                  series, entropic, walls)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
        ws_ptr = ws.data_ptr()
    sptr = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
    h = _vp()
    rc = lib().lbm_init(ctypes.byref(h), bx, len(boxes), ctypes.byref(op), *[_d(a) for a in arrs], sptr,
                        ws_ptr, ws_bytes)
    _check(rc, "lbm_init")
    return Context(h, boxes, ws, stream)


def init_device(boxes, rho, ux, uy, uz, theta, storage="f32", tau_conv=TAU_LB, rho0=1.0, newton_iters=0,
                shift_exp=None, stream=None, stochastic=False, seed=0, isothermal=False, series=False,
                entropic=False, walls=False):
    """lbm_init_device: the five fields are contiguous float64 torch CUDA
    tensors (all boxes concatenated); the equilibrium is built from them on
    the device. The workspace is a torch uint8 tensor held by the Context."""
    import torch
    bx = _boxes(boxes)
    op = _opts(storage, tau_conv, rho0, newton_iters, shift_exp, stochastic, seed, isothermal, series, entropic,
               walls)
    nodes = sum(2 * b[0] * b[1] * b[2] for b in boxes)
    fields = (rho, ux, uy, uz, theta)
    for a in fields:
        if not (isinstance(a, torch.Tensor) and a.is_cuda and a.dtype == torch.float64 and a.is_contiguous()):
            raise TypeError("init_device takes contiguous float64 CUDA tensors")
        if a.numel() != nodes:
            raise ValueError("field has %d values, boxes have %d nodes" % (a.numel(), nodes))
    ws_bytes = workspace_size(boxes, storage, tau_conv, rho0, newton_iters, shift_exp, stochastic, isothermal, series,
                              entropic, walls)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    sptr = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
    if stream is not None:
        # the fields were written on torch's current stream
        stream.wait_stream(torch.cuda.current_stream())
    h = _vp()
    rc = lib().lbm_init_device(ctypes.byref(h), bx, len(boxes), ctypes.byref(op), *[a.data_ptr() for a in fields],
                               sptr, ws.data_ptr(), ws_bytes)
    _check(rc, "lbm_init_device")
    return Context(h, boxes, ws, stream)


def selftest():
    return int(lib().lbm_selftest())


def collide_host(f, omega, precision="f32", newton=None, isothermal=False, series=False, entropic=False):
    """The kernel's per-node collision run on the host (FP64 or FP32)."""
    f = np.ascontiguousarray(f, dtype=np.float64).reshape(NQ)
    out = np.zeros(NQ)
    pr = {"f64": 0, "f32": 1}[precision]
    nt = (3 if pr == 0 else 1) if newton is None else int(newton)
    flags = ((FLAG_ISOTHERMAL if isothermal else 0) | (FLAG_SERIES_EQUILIBRIUM if series else 0)
             | (FLAG_ENTROPIC if entropic else 0))
    _check(lib().lbm_collide_host(pr, nt, flags, float(omega), _d(f), _d(out)),
           "lbm_collide_host")
    return out


def totals_noalloc(f_ptr, storage, dims, qstride, rho0=1.0, shift_exp=0, stream=None, out_ptr=None):
    """lbm_totals_noalloc: FP64 totals of one box held in caller device
    memory at f_ptr (populations [q][node], q-blocks qstride elements apart)
    into 5 doubles at the device pointer out_ptr, queued on `stream` (a
    torch.cuda.Stream, a raw handle or None)."""
    box = Box(int(dims[0]), int(dims[1]), int(dims[2]), 0, 0.0)
    h = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
    _check(lib().lbm_totals_noalloc(ctypes.c_void_p(int(f_ptr)), STORAGE[storage] if isinstance(storage, str)
                                    else int(storage), ctypes.byref(box), int(qstride), float(rho0), int(shift_exp),
                                    ctypes.c_void_p(h) if h else None, ctypes.c_void_p(int(out_ptr))),
           "lbm_totals_noalloc")


def device_copy(src_ptr, dst_ptr, nbytes, stream=None):
    """lbm_device_copy: the library's plain copy of nbytes bytes between
    device pointers (a measurement helper), queued on `stream` (a
    torch.cuda.Stream, a raw handle or None)."""
    h = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
    _check(lib().lbm_device_copy(ctypes.c_void_p(int(src_ptr)), ctypes.c_void_p(int(dst_ptr)), int(nbytes),
                                 ctypes.c_void_p(h) if h else None), "lbm_device_copy")


def tune_cache_file(path):
    """Back the process-wide tuning cache with a text file (None: in-process only)."""
    _check(lib().lbm_tune_cache_file(None if path is None else str(path).encode()), "lbm_tune_cache_file")


def tune_cache_clear():
    _check(lib().lbm_tune_cache_clear(), "lbm_tune_cache_clear")


def tune_cache_count():
    return int(lib().lbm_tune_cache_count())


def num_variants():
    return int(lib().lbm_num_variants())


def variant_desc(v):
    b = ctypes.c_int32(0)
    f = ctypes.c_uint32(0)
    _check(lib().lbm_variant_desc(int(v), ctypes.byref(b), ctypes.byref(f)), "lbm_variant_desc")
    return int(b.value), int(f.value)
