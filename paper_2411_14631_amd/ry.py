"""Python binding of the octree hydro C ABI (include/ry.h).

Argument marshalling only: every step of the hydro path runs in the HIP
library.  PyTorch provides the device memory (through the dev_alloc hook)
and the stream the library enqueues its work on.  If the compiled library
is missing this module raises on import of the library, it never falls back
to another implementation.
"""
from __future__ import annotations

import ctypes as C
import json
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# RY_DEBUG_LIB=1 loads the debug build (device index bounds checks that latch
# an error instead of accessing out of bounds; slower)
LIB_PATH = os.path.join(HERE, "libry_debug.so" if os.environ.get("RY_DEBUG_LIB") == "1" else "libry.so")

RY_OK, RY_EINVAL, RY_ENOMEM, RY_EHIP, RY_ESTATE, RY_ENUMERIC = 0, -1, -2, -3, -4, -5
RY_FP64, RY_MIXED = 0, 1
PRECISION = {"fp64": RY_FP64, "mixed": RY_MIXED}

# Every function declared in include/ry.h.
EXPORTS = [
    "ry_create", "ry_destroy", "ry_amr_build", "ry_level_info", "ry_get_mesh", "ry_cfl_dt",
    "ry_hydro_step", "ry_advance", "ry_conserved_totals", "ry_download", "ry_upload",
    "ry_batch_create", "ry_batch_run", "ry_batch_box_info", "ry_batch_download",
    "ry_set_tuning", "ry_get_tuning", "ry_set_level_tuning", "ry_get_level_tuning", "ry_autotune", "ry_floor_count", "ry_set_timing",
    "ry_kernel_time", "ry_cfl_dt_noalloc", "ry_copy_probe", "ry_last_error", "ry_mesh_build", "ry_mesh_level",
    "ry_mesh_free", "ry_hilbert_key", "ry_regrid", "ry_set_refine_param", "ry_set_regrid_device",
]
# Every function declared in include/ry_poisson.h.
POISSON_EXPORTS = [
    "ry_poisson_create", "ry_poisson_destroy", "ry_poisson_set_rhs", "ry_poisson_solve", "ry_poisson_iterate",
    "ry_poisson_eps_history", "ry_poisson_download", "ry_poisson_scalars", "ry_poisson_set_timing",
    "ry_poisson_kernel_time", "ry_poisson_last_error",
]
RY_PBC_PERIODIC, RY_PBC_DIRICHLET = 0, 1
RY_PC_NONE, RY_PC_STENCIL7 = 0, 1
POISSON_VECTORS = ("x", "r", "u", "w", "z", "q", "s", "p")

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
FILL_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_int32), C.POINTER(C.c_double))


class RyConfig(C.Structure):
    _fields_ = [("level_min", C.c_int32), ("level_max", C.c_int32), ("nbase", C.c_int32 * 3),
                ("boxlen", C.c_double), ("gamma", C.c_double), ("cfl", C.c_double),
                ("bc", C.c_int32 * 6), ("precision", C.c_int32), ("refine", C.c_int32),
                ("refine_param", C.c_double), ("rho_floor", C.c_double), ("p_floor", C.c_double),
                ("stream", C.c_void_p), ("dev_alloc", ALLOC_FN), ("dev_free", FREE_FN),
                ("alloc_user", C.c_void_p), ("nscalar", C.c_int32)]


class RyPoissonConfig(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("bc", C.c_int32), ("precond", C.c_int32), ("stream", C.c_void_p),
                ("dev_alloc", ALLOC_FN), ("dev_free", FREE_FN), ("alloc_user", C.c_void_p)]


class RyTuning(C.Structure):
    _fields_ = [("tiles_per_wg", C.c_int32), ("persistent", C.c_int32), ("waves_per_cu", C.c_int32),
                ("batch", C.c_int32), ("waves_per_tile", C.c_int32), ("tile_cells", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RyError(RuntimeError):
    def __init__(self, what, code, msg):
        super().__init__(f"{what} failed with status {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load the compiled library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "or python paper_2411_14631_amd/build.py")
    L = C.CDLL(LIB_PATH)
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "ry_create": ([C.POINTER(RyConfig), C.POINTER(P)], I32),
        "ry_destroy": ([P], None),
        "ry_amr_build": ([P, C.POINTER(D), FILL_FN, P], I32),
        "ry_level_info": ([P, I32, C.POINTER(I64), C.POINTER(I64)], I32),
        "ry_get_mesh": ([P, I32, P, P], I32),
        "ry_cfl_dt": ([P, C.POINTER(D)], I32),
        "ry_hydro_step": ([P, I32, D], I32),
        "ry_advance": ([P, I32, D, C.POINTER(D)], I32),
        "ry_conserved_totals": ([P, C.POINTER(D)], I32),
        "ry_download": ([P, I32, P], I32),
        "ry_upload": ([P, I32, P], I32),
        "ry_batch_create": ([C.POINTER(RyConfig), I32, C.POINTER(C.POINTER(D)), C.POINTER(P)], I32),
        "ry_batch_run": ([P, I32], I32),
        "ry_batch_box_info": ([P, I32, C.POINTER(I64), C.POINTER(D)], I32),
        "ry_batch_download": ([P, I32, P], I32),
        "ry_set_tuning": ([P, C.POINTER(RyTuning)], I32),
        "ry_get_tuning": ([P, C.POINTER(RyTuning)], I32),
        "ry_set_level_tuning": ([P, I32, C.POINTER(RyTuning)], I32),
        "ry_get_level_tuning": ([P, I32, C.POINTER(RyTuning)], I32),
        "ry_autotune": ([P, C.POINTER(RyTuning), C.POINTER(D), I32, C.POINTER(I32)], I32),
        "ry_floor_count": ([P], I64),
        "ry_set_timing": ([P, I32], I32),
        "ry_kernel_time": ([P, C.c_char_p, C.POINTER(I64), C.POINTER(D)], I32),
        "ry_copy_probe": ([P, C.c_size_t, I32, C.POINTER(D)], I32),
        "ry_last_error": ([P], C.c_char_p),
        "ry_mesh_build": ([C.POINTER(RyConfig), C.POINTER(D), FILL_FN, P, C.POINTER(P)], I32),
        "ry_mesh_level": ([P, I32, C.POINTER(I64), P, P, C.POINTER(I64)], I32),
        "ry_mesh_free": ([P], None),
        "ry_hilbert_key": ([I32, C.c_uint32, C.c_uint32, C.c_uint32], C.c_uint64),
        "ry_regrid": ([P, C.POINTER(I64), C.POINTER(I64)], I32),
        "ry_set_refine_param": ([P, D], I32),
        "ry_set_regrid_device": ([P, I32], I32),
        "ry_poisson_create": ([C.POINTER(RyPoissonConfig), C.POINTER(P)], I32),
        "ry_poisson_destroy": ([P], None),
        "ry_poisson_set_rhs": ([P, P, P], I32),
        "ry_poisson_solve": ([P, D, I32, C.POINTER(I32)], I32),
        "ry_poisson_iterate": ([P, I32], I32),
        "ry_poisson_eps_history": ([P, P, I32, C.POINTER(I32)], I32),
        "ry_poisson_download": ([P, I32, P], I32),
        "ry_poisson_scalars": ([P, C.POINTER(D), C.POINTER(D), C.POINTER(I32)], I32),
        "ry_poisson_set_timing": ([P, I32], I32),
        "ry_poisson_kernel_time": ([P, C.POINTER(I32), C.POINTER(D)], I32),
        "ry_poisson_last_error": ([P], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


class _TorchMemory:
    """dev_alloc / dev_free hooks backed by torch's caching allocator."""

    def __init__(self, torch, device):
        self.torch = torch
        self.device = device
        self.live = {}

        def alloc(nbytes, user):
            try:
                t = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device=self.device)
            except RuntimeError:
                return None
            p = t.data_ptr()
            self.live[p] = t
            return p

        def free(p, user):
            self.live.pop(p, None)

        self.alloc_cb = ALLOC_FN(alloc)
        self.free_cb = FREE_FN(free)

    def bytes(self):
        return sum(t.numel() for t in self.live.values())


def _make_fill(fill, nv=5):
    def cb(user, level, ncell, ijk, U):
        a = np.ctypeslib.as_array(ijk, shape=(ncell, 3)).copy()
        out = np.ctypeslib.as_array(U, shape=(nv, ncell))
        out[...] = fill(int(level), a)
    return FILL_FN(cb)


def _config(prob, precision, stream_handle, mem):
    cfg = RyConfig()
    cfg.level_min, cfg.level_max = prob.level_min, prob.level_max
    for a in range(3):
        cfg.nbase[a] = prob.nbase[a]
    cfg.boxlen, cfg.gamma, cfg.cfl = prob.boxlen, prob.gamma, prob.cfl
    for i in range(6):
        cfg.bc[i] = prob.bc[i]
    cfg.precision = PRECISION[precision]
    cfg.refine, cfg.refine_param = prob.refine, prob.refine_param
    cfg.rho_floor, cfg.p_floor = prob.rho_floor, prob.p_floor
    cfg.nscalar = getattr(prob, "nscalar", 0)
    cfg.stream = stream_handle
    if mem is not None:
        cfg.dev_alloc = mem.alloc_cb
        cfg.dev_free = mem.free_cb
    return cfg


def _read_json(path):
    """The tuning cache (an empty one when the file does not exist yet)."""
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


class _Base:
    def _check(self, rc, what):
        if rc != RY_OK:
            msg = lib().ry_last_error(self.ctx).decode() if self.ctx else ""
            raise RyError(what, rc, msg)

    def close(self):
        if getattr(self, "ctx", None) and self.ctx.value:
            lib().ry_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # tuning / timing / diagnostics
    def set_tuning(self, tiles_per_wg=1, persistent=0, waves_per_cu=4, batch=1, waves_per_tile=1, tile_cells=4):
        t = RyTuning(tiles_per_wg, persistent, waves_per_cu, batch, waves_per_tile, tile_cells)
        self._check(lib().ry_set_tuning(self.ctx, C.byref(t)), "ry_set_tuning")

    def tuning(self):
        t = RyTuning()
        self._check(lib().ry_get_tuning(self.ctx, C.byref(t)), "ry_get_tuning")
        return t.as_dict()

    def set_level_tuning(self, level, tiles_per_wg=1, persistent=0, waves_per_cu=4, batch=1, waves_per_tile=1,
                         tile_cells=4):
        t = RyTuning(tiles_per_wg, persistent, waves_per_cu, batch, waves_per_tile, tile_cells)
        self._check(lib().ry_set_level_tuning(self.ctx, level, C.byref(t)), "ry_set_level_tuning")

    def level_tuning(self, level):
        t = RyTuning()
        self._check(lib().ry_get_level_tuning(self.ctx, level, C.byref(t)), "ry_get_level_tuning")
        return t.as_dict()

    def autotune(self, cache=None):
        """Time the launch candidates and keep the fastest per level
        (ry_autotune): (level-0 tuning, per-candidate times).  With `cache`,
        a JSON file: a result stored there for the same workload (its mesh),
        precision and GPU architecture is applied without timing (times are
        then empty); a new result is added to the file."""
        key = self._tune_key() if cache else None
        if key:
            stored = _read_json(cache).get(key)
            if stored:
                for lv, t in zip(self._tune_levels(), stored):
                    self._apply_level_tuning(lv, t)
                return self._first_tuning(), []
        best = RyTuning()
        times = (C.c_double * 64)()
        n = C.c_int32()
        self._check(lib().ry_autotune(self.ctx, C.byref(best), times, 64, C.byref(n)), "ry_autotune")
        if key:
            d = _read_json(cache)
            d[key] = [self._level_tuning_of(lv) for lv in self._tune_levels()]
            tmp = f"{cache}.{os.getpid()}.tmp"
            with open(tmp, "w") as f:
                json.dump(d, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return best.as_dict(), list(times[: n.value])

    def _arch(self):
        return self.torch.cuda.get_device_properties(self.torch.cuda.current_device()).gcnArchName

    # the tuned levels and their tunings (a batch context has one)
    def _tune_levels(self):
        return [None]

    def _level_tuning_of(self, lv):
        return self.tuning()

    def _apply_level_tuning(self, lv, t):
        self.set_tuning(**t)

    def _first_tuning(self):
        return self.tuning()

    def set_timing(self, on=True):
        self._check(lib().ry_set_timing(self.ctx, 1 if on else 0), "ry_set_timing")

    def kernel_time(self, name="hydro"):
        n = C.c_int64()
        ms = C.c_double()
        self._check(lib().ry_kernel_time(self.ctx, name.encode(), C.byref(n), C.byref(ms)), "ry_kernel_time")
        return n.value, ms.value

    def floors(self):
        return lib().ry_floor_count(self.ctx)

    def copy_probe(self, nbytes, reps=20):
        ms = C.c_double()
        self._check(lib().ry_copy_probe(self.ctx, nbytes, reps, C.byref(ms)), "ry_copy_probe")
        return ms.value


class Hydro(_Base):
    """One octree (uniform or AMR) on the GPU, built from a workloads.Problem."""

    def __init__(self, prob, precision="fp64", device="cuda", torch_memory=True, memory=None):
        import torch
        self.torch = torch
        self.prob = prob
        self.ctx = C.c_void_p()
        self.stream = torch.cuda.Stream(device=device)       # default priority
        # device memory: torch's caching allocator (default), a caller-supplied
        # object with alloc_cb / free_cb, or hipMalloc (torch_memory=False)
        self.mem = memory if memory is not None else (_TorchMemory(torch, device) if torch_memory else None)
        cfg = _config(prob, precision, self.stream.cuda_stream, self.mem)
        self._cfg = cfg
        self._check(lib().ry_create(C.byref(cfg), C.byref(self.ctx)), "ry_create")
        base = prob.base_flat()
        nv = self.nv = 5 + prob.nscalar
        self._fill = _make_fill(prob.fill if prob.fill else (lambda l, ijk: np.zeros((nv, len(ijk)))), nv)
        self._check(lib().ry_amr_build(self.ctx, base.ctypes.data_as(C.POINTER(C.c_double)), self._fill, None),
                    "ry_amr_build")
        self.t = 0.0

    @property
    def levels(self):
        return range(self.prob.level_min, self.prob.level_max + 1)

    def _tune_key(self):
        mesh = [self.level_info(lv) for lv in self.levels]
        prec = "mixed" if self._cfg.precision == RY_MIXED else "fp64"
        return f"{self.prob.name}|{mesh}|{prec}|{self._arch()}"

    def _tune_levels(self):
        return list(self.levels)

    def _level_tuning_of(self, lv):
        return self.level_tuning(lv)

    def _apply_level_tuning(self, lv, t):
        self.set_level_tuning(lv, **t)

    def _first_tuning(self):
        return self.level_tuning(self.prob.level_min)

    def level_info(self, level):
        n, leaf = C.c_int64(), C.c_int64()
        self._check(lib().ry_level_info(self.ctx, level, C.byref(n), C.byref(leaf)), "ry_level_info")
        return n.value, leaf.value

    def mesh(self, level):
        n, _ = self.level_info(level)
        keys = np.zeros(n, np.uint64)
        ref = np.zeros(n, np.uint8)
        self._check(lib().ry_get_mesh(self.ctx, level, keys.ctypes.data, ref.ctypes.data), "ry_get_mesh")
        return keys, ref

    def download(self, level):
        n, _ = self.level_info(level)
        U = np.zeros((self.nv, 8 * n), np.float64)
        self._check(lib().ry_download(self.ctx, level, U.ctypes.data), "ry_download")
        return U

    def upload(self, level, U):
        U = np.ascontiguousarray(U, np.float64)
        self._check(lib().ry_upload(self.ctx, level, U.ctypes.data), "ry_upload")

    def cfl_dt(self):
        dt = C.c_double()
        self._check(lib().ry_cfl_dt(self.ctx, C.byref(dt)), "ry_cfl_dt")
        return dt.value

    def hydro_step(self, level, dt):
        self._check(lib().ry_hydro_step(self.ctx, level, dt), "ry_hydro_step")

    def coarse_step(self, dt):
        """Fine-first recursion of one coarse step through ry_hydro_step."""
        def rec(level, d):
            if level < self.prob.level_max and self.level_info(level + 1)[0] > 0:
                rec(level + 1, 0.5 * d)
                rec(level + 1, 0.5 * d)
            self.hydro_step(level, d)
        rec(self.prob.level_min, dt)

    def advance(self, n_coarse, t_end=math.inf):
        t = C.c_double(self.t)
        self._check(lib().ry_advance(self.ctx, n_coarse, t_end, C.byref(t)), "ry_advance")
        self.t = t.value

    def regrid(self):
        """Dynamic refinement between coarse steps: (octs created, destroyed)."""
        a, b = C.c_int64(), C.c_int64()
        self._check(lib().ry_regrid(self.ctx, C.byref(a), C.byref(b)), "ry_regrid")
        return a.value, b.value

    def set_refine_param(self, value):
        self._check(lib().ry_set_refine_param(self.ctx, value), "ry_set_refine_param")

    def set_regrid_device(self, on):
        """True (default): regrid entirely on the device; False: flags and
        tables on the host, state remap on the device."""
        self._check(lib().ry_set_regrid_device(self.ctx, 1 if on else 0), "ry_set_regrid_device")

    def totals(self):
        tot = (C.c_double * self.nv)()
        self._check(lib().ry_conserved_totals(self.ctx, tot), "ry_conserved_totals")
        return np.array(tot[:])


class BatchHydro(_Base):
    """Many independent single-level boxes advanced together."""

    def __init__(self, probs, precision="fp64", device="cuda", torch_memory=True):
        import torch
        self.torch = torch
        self.probs = probs
        self._precision = precision
        self.ctx = C.c_void_p()
        self.stream = torch.cuda.Stream(device=device)
        self.mem = _TorchMemory(torch, device) if torch_memory else None
        n = len(probs)
        cfgs = (RyConfig * n)(*[_config(p, precision, self.stream.cuda_stream, self.mem) for p in probs])
        self._bases = [p.base_flat() for p in probs]
        ptrs = (C.POINTER(C.c_double) * n)(*[b.ctypes.data_as(C.POINTER(C.c_double)) for b in self._bases])
        self._check(lib().ry_batch_create(cfgs, n, ptrs, C.byref(self.ctx)), "ry_batch_create")
        self._bases = None

    def run(self, nsteps):
        self._check(lib().ry_batch_run(self.ctx, nsteps), "ry_batch_run")

    def _tune_key(self):
        import hashlib
        names = hashlib.sha256("|".join(p.name for p in self.probs).encode()).hexdigest()[:16]
        return f"batch{len(self.probs)}:{names}|{self._precision}|{self._arch()}"

    def box_info(self, b):
        n, t = C.c_int64(), C.c_double()
        self._check(lib().ry_batch_box_info(self.ctx, b, C.byref(n), C.byref(t)), "ry_batch_box_info")
        return n.value, t.value

    def download(self, b):
        n, _ = self.box_info(b)
        U = np.zeros((5, 8 * n), np.float64)
        self._check(lib().ry_batch_download(self.ctx, b, U.ctypes.data), "ry_batch_download")
        return U


class HostMesh:
    """The library's own octree builder run on the host (no GPU needed)."""

    def __init__(self, prob):
        self.prob = prob
        self.m = C.c_void_p()
        cfg = _config(prob, "fp64", None, None)
        base = prob.base_flat()
        nv = 5 + prob.nscalar
        self._fill = _make_fill(prob.fill if prob.fill else (lambda l, ijk: np.zeros((nv, len(ijk)))), nv)
        rc = lib().ry_mesh_build(C.byref(cfg), base.ctypes.data_as(C.POINTER(C.c_double)), self._fill, None,
                                 C.byref(self.m))
        if rc != RY_OK:
            raise RyError("ry_mesh_build", rc, "")

    def level(self, level):
        n, ng = C.c_int64(), C.c_int64()
        if lib().ry_mesh_level(self.m, level, C.byref(n), None, None, C.byref(ng)) != RY_OK:
            raise RyError("ry_mesh_level", RY_EINVAL, "")
        keys = np.zeros(n.value, np.uint64)
        ref = np.zeros(n.value, np.uint8)
        lib().ry_mesh_level(self.m, level, C.byref(n), keys.ctypes.data, ref.ctypes.data, C.byref(ng))
        return keys, ref, ng.value

    def __del__(self):
        if getattr(self, "m", None) and self.m.value:
            lib().ry_mesh_free(self.m)
            self.m = C.c_void_p()


def hilbert_key(bits, x, y, z):
    return lib().ry_hilbert_key(bits, x, y, z)


def create_status(prob, precision="fp64"):
    """ry_create's status for a problem (validation runs before any device
    call, so invalid configurations are rejected without a GPU)."""
    cfg = _config(prob, precision, None, None)
    ctx = C.c_void_p()
    rc = lib().ry_create(C.byref(cfg), C.byref(ctx))
    if rc == RY_OK:
        lib().ry_destroy(ctx)
    return rc


def _poisson_config(shape, bc, precond, stream_handle, mem):
    """shape = (n2, n1, n0) of a numpy grid array (x fastest)."""
    cfg = RyPoissonConfig()
    cfg.n[0], cfg.n[1], cfg.n[2] = int(shape[2]), int(shape[1]), int(shape[0])
    cfg.bc, cfg.precond = bc, precond
    cfg.stream = stream_handle
    if mem is not None:
        cfg.dev_alloc = mem.alloc_cb
        cfg.dev_free = mem.free_cb
    return cfg


class Poisson:
    """PPCG Poisson solver on one uniform grid (include/ry_poisson.h).

    Grid arrays are numpy arrays of shape (n2, n1, n0), x fastest."""

    def __init__(self, shape, bc=RY_PBC_PERIODIC, precond=RY_PC_STENCIL7, device="cuda", torch_memory=True):
        import torch
        self.torch = torch
        self.shape = tuple(int(v) for v in shape)
        self.ctx = C.c_void_p()
        self.stream = torch.cuda.Stream(device=device)       # default priority
        self.mem = _TorchMemory(torch, device) if torch_memory else None
        cfg = _poisson_config(self.shape, bc, precond, self.stream.cuda_stream, self.mem)
        self._cfg = cfg
        self._check(lib().ry_poisson_create(C.byref(cfg), C.byref(self.ctx)), "ry_poisson_create")

    def _check(self, rc, what):
        if rc != RY_OK:
            msg = lib().ry_poisson_last_error(self.ctx).decode() if self.ctx else ""
            raise RyError(what, rc, msg)

    def close(self):
        if getattr(self, "ctx", None) and self.ctx.value:
            lib().ry_poisson_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _grid(self, a):
        a = np.ascontiguousarray(a, np.float64)
        if a.shape != self.shape:
            raise ValueError(f"grid array of shape {a.shape}, solver shape {self.shape}")
        return a

    def set_rhs(self, b, x0=None):
        self._b = self._grid(b)
        self._x0 = None if x0 is None else self._grid(x0)
        self._check(lib().ry_poisson_set_rhs(self.ctx, self._b.ctypes.data,
                                             None if self._x0 is None else self._x0.ctypes.data),
                    "ry_poisson_set_rhs")

    def solve(self, eps=1e-4, max_iter=1000):
        n = C.c_int32()
        self._check(lib().ry_poisson_solve(self.ctx, eps, max_iter, C.byref(n)), "ry_poisson_solve")
        return n.value

    def iterate(self, n):
        self._check(lib().ry_poisson_iterate(self.ctx, n), "ry_poisson_iterate")

    def eps_history(self):
        buf = np.zeros(65536)
        n = C.c_int32()
        self._check(lib().ry_poisson_eps_history(self.ctx, buf.ctypes.data, len(buf), C.byref(n)),
                    "ry_poisson_eps_history")
        return buf[: n.value].copy()

    def download(self, which="x"):
        out = np.zeros(self.shape)
        self._check(lib().ry_poisson_download(self.ctx, POISSON_VECTORS.index(which), out.ctypes.data),
                    "ry_poisson_download")
        return out

    def state(self):
        """All eight recurrence vectors plus (alpha_prev, gamma_prev, i)."""
        a, g, i = C.c_double(), C.c_double(), C.c_int32()
        self._check(lib().ry_poisson_scalars(self.ctx, C.byref(a), C.byref(g), C.byref(i)), "ry_poisson_scalars")
        return {k: self.download(k) for k in POISSON_VECTORS}, a.value, g.value, i.value

    def set_timing(self, on=True):
        self._check(lib().ry_poisson_set_timing(self.ctx, 1 if on else 0), "ry_poisson_set_timing")

    def kernel_time(self):
        n, ms = C.c_int32(), C.c_double()
        self._check(lib().ry_poisson_kernel_time(self.ctx, C.byref(n), C.byref(ms)), "ry_poisson_kernel_time")
        return n.value, ms.value


def poisson_create_status(shape, bc=RY_PBC_PERIODIC, precond=RY_PC_STENCIL7):
    """ry_poisson_create's status (validation runs before any device call)."""
    cfg = _poisson_config(shape, bc, precond, None, None)
    ctx = C.c_void_p()
    rc = lib().ry_poisson_create(C.byref(cfg), C.byref(ctx))
    if rc == RY_OK:
        lib().ry_poisson_destroy(ctx)
    return rc
