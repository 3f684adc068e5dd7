"""Python binding of libnncert (ctypes): argument marshalling only.

Every step of the maintenance path runs in the library's HIP kernels.  PyTorch
is used for device memory and streams: callers pass contiguous CUDA tensors and
the binding hands their data pointers and the current stream to the C ABI.

torch must be imported before the library is loaded so that both use the one
HIP runtime that torch ships (they share its soname); this module does so.
If the built library is missing, loading raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnncert.so")

NNC_OK = 0
NNC_E_INVAL = -1
NNC_E_NOMEM = -2
NNC_E_HIP = -3
NNC_E_EPS = -4
NNC_E_NONFINITE = -5
NNC_E_STATE = -6
NNC_E_DEVICE = -7

NNC_COPY_POSITIONS = 1
NNC_SYNC = 2
NNC_QUERY_TILED = 4
NNC_QUERY_POINTWISE = 8
NNC_BUDGET = 16
NNC_QUEUE = 32

NNC_FAILED = 0
NNC_CANDIDATES = 1

EXPORTS = (
    "nnc_create", "nnc_destroy", "nnc_init_certificates", "nnc_step", "nnc_repair", "nnc_rebuild",
    "nnc_oracle_verify", "nnc_rho_predict", "nnc_frontier_entropy", "nnc_get_state", "nnc_snapshot", "nnc_restore",
    "nnc_snap_free", "nnc_allpairs_top2", "nnc_strerror", "nnc_profile_enable", "nnc_profile_read",
    "nnc_batch_create", "nnc_batch_destroy", "nnc_batch_offsets", "nnc_batch_init", "nnc_batch_step",
    "nnc_batch_selector_load", "nnc_batch_scene_stats", "nnc_batch_get_state", "nnc_features",
    "nnc_mlp_workspace_bytes", "nnc_mlp_grad", "nnc_mlp_adam", "nnc_mlp_forward", "nnc_snapshot_update",
    "nnc_sqrt_f32", "nnc_mlp_grad_static", "nnc_frontier_gyration", "nnc_queue_stats",
    "nnc_batch_snapshot", "nnc_batch_restore", "nnc_batch_snap_free", "nnc_batch_snapshot_update",
    "nnc_batch_selector_band",
)

POLICY_REPAIR, POLICY_REBUILD, POLICY_THRESHOLD, POLICY_LEARNED = range(4)
NFEATURES = 6
SELECTOR_PARAMS = 4738

K_INGEST, K_FILTER, K_GRID, K_QUERY, K_ENTROPY = range(5)
KERNEL_CLASSES = ("ingest", "filter", "grid", "query", "entropy")


class NNCError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


class Config(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("grid_g", ctypes.c_int32), ("n", ctypes.c_int64),
                ("guard", ctypes.c_double), ("refresh", ctypes.c_double), ("stream", ctypes.c_void_p),
                ("flags", ctypes.c_uint32), ("block", ctypes.c_int32),
                ("lo", ctypes.c_float * 3), ("hi", ctypes.c_float * 3)]


class Frontier(ctypes.Structure):
    _fields_ = [("idx_dev", ctypes.c_void_p), ("count_dev", ctypes.c_void_p),
                ("count_host", ctypes.c_int32), ("step", ctypes.c_int32)]


class State(ctypes.Structure):
    _fields_ = [("nn", ctypes.c_void_p), ("d1", ctypes.c_void_p), ("d2", ctypes.c_void_p),
                ("e", ctypes.c_void_p), ("cell", ctypes.c_void_p), ("fail", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("d", ctypes.c_int32), ("grid_g", ctypes.c_int32),
                ("rho", ctypes.c_void_p), ("Si", ctypes.c_void_p)]


class Audit(ctypes.Structure):
    _fields_ = [("n_checked", ctypes.c_int64), ("n_detect", ctypes.c_int64), ("n_true_fail", ctypes.c_int64),
                ("n_missed", ctypes.c_int64), ("n_false", ctypes.c_int64), ("n_value_mismatch", ctypes.c_int64),
                ("nn_hash", ctypes.c_uint64), ("rho_flagged", ctypes.c_int64), ("rho_hit", ctypes.c_int64)]


class Entropy(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("S", ctypes.c_double), ("H", ctypes.c_double),
                ("m", ctypes.c_int32), ("C", ctypes.c_int32), ("count", ctypes.c_int32)]


class Profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 5), ("count", ctypes.c_int64 * 5)]


class BatchConfig(ctypes.Structure):
    _fields_ = [("scenes", ctypes.c_int32), ("n", ctypes.c_void_p), ("d", ctypes.c_void_p),
                ("grid_g", ctypes.c_void_p), ("lanes", ctypes.c_int32), ("guard", ctypes.c_double),
                ("refresh", ctypes.c_double), ("stream", ctypes.c_void_p), ("flags", ctypes.c_uint32)]


class SceneStats(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("S", ctypes.c_double), ("H_fail", ctypes.c_double),
                ("H_cand", ctypes.c_double), ("n_cand", ctypes.c_int32), ("n_fail", ctypes.c_int32),
                ("m_cand", ctypes.c_int32), ("C", ctypes.c_int32), ("strategy", ctypes.c_int32),
                ("err", ctypes.c_int32), ("features", ctypes.c_float * 6),
                ("t_filter_us", ctypes.c_double), ("t_grid_us", ctypes.c_double), ("t_query_us", ctypes.c_double)]


_lib = None
_hip = None


def load():
    """Load libnncert.so (built in-tree); raises if it has not been built."""
    global _lib, _hip
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                           f"or python paper_2606_18314_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    lib.nnc_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(Config)]
    lib.nnc_destroy.argtypes = [P]
    lib.nnc_destroy.restype = None
    lib.nnc_init_certificates.argtypes = [P, P]
    lib.nnc_step.argtypes = [P, P, ctypes.c_float, ctypes.POINTER(Frontier)]
    lib.nnc_repair.argtypes = [P, ctypes.POINTER(Frontier)]
    lib.nnc_rebuild.argtypes = [P]
    lib.nnc_oracle_verify.argtypes = [P, ctypes.POINTER(Audit)]
    lib.nnc_rho_predict.argtypes = [P]
    lib.nnc_frontier_entropy.argtypes = [P, ctypes.c_int, ctypes.POINTER(Entropy)]
    lib.nnc_get_state.argtypes = [P, ctypes.POINTER(State)]
    lib.nnc_snapshot.argtypes = [P, ctypes.POINTER(P)]
    lib.nnc_restore.argtypes = [P, P]
    lib.nnc_snapshot_update.argtypes = [P, P]
    lib.nnc_snap_free.argtypes = [P]
    lib.nnc_snap_free.restype = None
    lib.nnc_allpairs_top2.argtypes = [P, ctypes.c_int64, ctypes.c_int32, P, ctypes.c_int64, P, P, P, P]
    lib.nnc_profile_enable.argtypes = [P, ctypes.c_int]
    lib.nnc_profile_read.argtypes = [P, ctypes.POINTER(Profile), ctypes.c_int]
    lib.nnc_batch_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(BatchConfig)]
    lib.nnc_batch_destroy.argtypes = [P]
    lib.nnc_batch_destroy.restype = None
    lib.nnc_batch_offsets.argtypes = [P, P, P]
    lib.nnc_batch_init.argtypes = [P, P]
    lib.nnc_batch_step.argtypes = [P, P, ctypes.c_int, ctypes.c_float]
    lib.nnc_batch_selector_load.argtypes = [P, P]
    lib.nnc_batch_scene_stats.argtypes = [P, P]
    lib.nnc_batch_get_state.argtypes = [P, ctypes.POINTER(State)]
    lib.nnc_features.argtypes = [P, P]
    lib.nnc_mlp_workspace_bytes.argtypes = [ctypes.c_int]
    lib.nnc_mlp_workspace_bytes.restype = ctypes.c_size_t
    lib.nnc_mlp_grad.argtypes = [P, P, P, P, ctypes.c_int, P, P, P, P]
    lib.nnc_mlp_grad_static.argtypes = [P, P, P, P, ctypes.c_int, P, P, P]
    lib.nnc_mlp_adam.argtypes = [P, P, P, P, ctypes.c_int, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                 ctypes.c_float, P]
    lib.nnc_mlp_forward.argtypes = [P, P, ctypes.c_int, P, P]
    lib.nnc_sqrt_f32.argtypes = [P, P, ctypes.c_int64, P]
    lib.nnc_queue_stats.argtypes = [P, ctypes.POINTER(ctypes.c_int64)]
    lib.nnc_batch_snapshot.argtypes = [P, ctypes.POINTER(P)]
    lib.nnc_batch_restore.argtypes = [P, P]
    lib.nnc_batch_snapshot_update.argtypes = [P, P]
    lib.nnc_batch_selector_band.argtypes = [P, ctypes.c_float, ctypes.c_float]
    lib.nnc_batch_snap_free.argtypes = [P]
    lib.nnc_batch_snap_free.restype = None
    lib.nnc_frontier_gyration.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double)]
    lib.nnc_strerror.argtypes = [ctypes.c_int]
    lib.nnc_strerror.restype = ctypes.c_char_p
    _lib = lib
    return lib


def hip():
    """The HIP runtime torch loaded (same soname), for raw device copies."""
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so.7")
        _hip.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                        ctypes.c_void_p]
    return _hip


def strerror(code: int) -> str:
    return load().nnc_strerror(code).decode()


def check(code: int, where: str) -> None:
    if code != NNC_OK:
        raise NNCError(code, where)


def _ptr(t) -> int:
    if t is None:
        return 0
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous CUDA tensor")
    return t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def copy_from_device(dst: torch.Tensor, src_ptr: int, nbytes: int, stream: int | None = None) -> torch.Tensor:
    """Copy nbytes of library-owned device memory into a CUDA tensor, ordered on ``stream``."""
    if nbytes:
        s = _stream() if stream is None else stream
        rc = hip().hipMemcpyAsync(dst.data_ptr(), src_ptr, nbytes, 3, s)  # 3 = device to device
        if rc != 0:
            raise RuntimeError(f"hipMemcpyAsync failed ({rc})")
    return dst


def copy_to_device(dst_ptr: int, src: torch.Tensor, stream: int | None = None) -> None:
    """Copy a contiguous CUDA tensor into library-owned device memory at dst_ptr, ordered on ``stream``."""
    nbytes = src.numel() * src.element_size()
    if nbytes:
        s = _stream() if stream is None else stream
        rc = hip().hipMemcpyAsync(dst_ptr, _ptr(src), nbytes, 3, s)
        if rc != 0:
            raise RuntimeError(f"hipMemcpyAsync failed ({rc})")


def allpairs_top2(pos: torch.Tensor, qidx: torch.Tensor | None = None):
    """Exact all-pairs top-2 of float32 [d, n] positions: (nn, d1, d2) CUDA tensors."""
    d, n = pos.shape
    nq = n if qidx is None else qidx.numel()
    dev = pos.device
    nn = torch.empty(nq, dtype=torch.int32, device=dev)
    d1 = torch.empty(nq, dtype=torch.float32, device=dev)
    d2 = torch.empty(nq, dtype=torch.float32, device=dev)
    check(load().nnc_allpairs_top2(_ptr(pos), n, d, _ptr(qidx), nq, _ptr(nn), _ptr(d1), _ptr(d2), _stream()),
          "nnc_allpairs_top2")
    return nn, d1, d2


def sqrt_f32(x: torch.Tensor) -> torch.Tensor:
    """Elementwise square root of a float32 CUDA tensor by the certificates' routine."""
    out = torch.empty_like(x)
    check(load().nnc_sqrt_f32(_ptr(x), _ptr(out), x.numel(), _stream()), "nnc_sqrt_f32")
    return out


class Snapshot:
    def __init__(self, handle: int):
        self.handle = handle

    def __del__(self):
        if self.handle and _lib is not None:
            _lib.nnc_snap_free(self.handle)
            self.handle = 0


class NNCert:
    """One moving point set and its certificates, on the current CUDA stream."""

    def __init__(self, n: int, d: int, grid_g: int = 0, guard: float = -1.0, refresh: float = 0.0,
                 copy_positions: bool = False, sync: bool = False, stream: int | None = None, lanes: int = 0,
                 all_query: str = "auto", box=None, budget: bool = False, queue: bool = False):
        """lanes: lanes per query (1, 4 (plane only), 8, 16, 32 or 64; 0 = 32 in the cube,
        16 in the plane).
        all_query: "auto", "tiled" or "pointwise" -- how initialisation and rebuild
        query every point (under "auto" tiled by cells from N = 65536 on at
        initialisation, from 2^17 (d = 2) or 2^19 (d = 3) on at a rebuild).
        box: (lo, hi), per-axis bounds of the grid's domain (default the unit box).
        budget: the per-point motion budget (NNC_BUDGET) tightens the candidate set.
        queue: the expiry calendar queue (NNC_QUEUE) replaces the filter's scan of all keys."""
        if all_query not in ("auto", "tiled", "pointwise"):
            raise ValueError("all_query: 'auto', 'tiled' or 'pointwise'")
        lib = load()
        self.n, self.d = int(n), int(d)
        self.stream = _stream() if stream is None else stream
        cfg = Config(d=self.d, grid_g=int(grid_g), n=self.n, guard=float(guard), refresh=float(refresh),
                     stream=self.stream,
                     flags=(NNC_COPY_POSITIONS if copy_positions else 0) | (NNC_SYNC if sync else 0)
                     | (NNC_QUERY_TILED if all_query == "tiled" else 0)
                     | (NNC_QUERY_POINTWISE if all_query == "pointwise" else 0)
                     | (NNC_BUDGET if budget else 0) | (NNC_QUEUE if queue else 0),
                     block=int(lanes))
        if box is not None:
            lo, hi = box
            for k in range(self.d):
                cfg.lo[k] = float(lo[k])
                cfg.hi[k] = float(hi[k])
        h = ctypes.c_void_p()
        check(lib.nnc_create(ctypes.byref(h), ctypes.byref(cfg)), "nnc_create")
        self.h = h.value
        self._keep = []  # borrowed position tensors stay alive while referenced by the library
        st = State()
        check(lib.nnc_get_state(self.h, ctypes.byref(st)), "nnc_get_state")
        self.grid_g = st.grid_g
        self._state = st
        self.frontier = Frontier()

    def close(self):
        # at interpreter exit the module globals may already be gone: then the process
        # is ending and its device memory with it
        if getattr(self, "h", None) and _lib is not None:
            _lib.nnc_destroy(self.h)
        self.h = None

    def __del__(self):
        self.close()

    def _hold(self, pos):
        self._keep = (self._keep + [pos])[-2:]

    def init_certificates(self, pos: torch.Tensor) -> None:
        self._hold(pos)
        check(_lib.nnc_init_certificates(self.h, _ptr(pos)), "nnc_init_certificates")

    def step(self, pos: torch.Tensor, eps_declared: float = -1.0) -> Frontier:
        self._hold(pos)
        check(_lib.nnc_step(self.h, _ptr(pos), float(eps_declared), ctypes.byref(self.frontier)), "nnc_step")
        return self.frontier

    def repair(self, idx: torch.Tensor | None = None, count: torch.Tensor | None = None) -> None:
        if idx is None:
            check(_lib.nnc_repair(self.h, None), "nnc_repair")
        else:
            f = Frontier(idx_dev=_ptr(idx), count_dev=_ptr(count), count_host=-1, step=0)
            check(_lib.nnc_repair(self.h, ctypes.byref(f)), "nnc_repair")

    def rebuild(self) -> None:
        check(_lib.nnc_rebuild(self.h), "nnc_rebuild")

    def oracle_verify(self) -> dict:
        a = Audit()
        check(_lib.nnc_oracle_verify(self.h, ctypes.byref(a)), "nnc_oracle_verify")
        return {k: getattr(a, k) for k, _ in Audit._fields_}

    def rho_predict(self) -> None:
        """The local failure predictor (audit only), between step and repair/rebuild."""
        check(_lib.nnc_rho_predict(self.h), "nnc_rho_predict")

    def frontier_entropy(self, which: int = NNC_FAILED) -> dict:
        e = Entropy()
        check(_lib.nnc_frontier_entropy(self.h, which, ctypes.byref(e)), "nnc_frontier_entropy")
        return {k: getattr(e, k) for k, _ in Entropy._fields_}

    def queue_stats(self) -> dict:
        """Work counters of the expiry calendar (NNC_QUEUE contexts)."""
        v = (ctypes.c_int64 * 6)()
        check(_lib.nnc_queue_stats(self.h, v), "nnc_queue_stats")
        return dict(zip(("pops", "full_scans", "builds", "entries_read", "pool_used", "far_keys"), list(v)))

    def frontier_gyration(self, which: int = NNC_FAILED):
        """(radius of gyration, centroid (x, y, z)) of the failed set or the candidates."""
        g = ctypes.c_double()
        cen = (ctypes.c_double * 3)()
        check(_lib.nnc_frontier_gyration(self.h, which, ctypes.byref(g), cen), "nnc_frontier_gyration")
        return g.value, tuple(cen)

    def frontier_indices(self) -> torch.Tensor:
        """The last step's candidate list as a CUDA int32 tensor (synchronises)."""
        cnt = torch.empty(1, dtype=torch.int32, device="cuda")
        copy_from_device(cnt, self.frontier.count_dev, 4, self.stream)
        torch.cuda.synchronize()
        k = int(cnt.item())
        out = torch.empty(k, dtype=torch.int32, device="cuda")
        copy_from_device(out, self.frontier.idx_dev, 4 * k, self.stream)
        torch.cuda.synchronize()
        return out

    def state(self) -> dict:
        """Copies of the state arrays as CUDA tensors."""
        st, n = self._state, self.n
        spec = [("nn", torch.int32, 4), ("d1", torch.float32, 4), ("d2", torch.float32, 4),
                ("e", torch.float64, 8), ("cell", torch.int32, 4), ("fail", torch.uint8, 1),
                ("Si", torch.float64, 8)]
        out = {}
        for name, dt, sz in spec:
            t = torch.empty(n, dtype=dt, device="cuda")
            out[name] = copy_from_device(t, getattr(st, name), n * sz, self.stream)
        torch.cuda.synchronize()
        return out

    def rho_flags(self) -> torch.Tensor:
        """Per-point flags of the last nnc_rho_predict (CUDA uint8 tensor)."""
        t = torch.empty(self.n, dtype=torch.uint8, device="cuda")
        copy_from_device(t, self._state.rho, self.n, self.stream)
        torch.cuda.synchronize()
        return t

    def state_pointers(self) -> dict:
        """Raw device addresses of the state arrays (nnc_get_state)."""
        st = State()
        check(_lib.nnc_get_state(self.h, ctypes.byref(st)), "nnc_get_state")
        return {k: getattr(st, k) for k, _ in State._fields_}

    def features(self) -> torch.Tensor:
        """The six selector features of the pending step (CUDA float32 tensor)."""
        out = torch.empty(NFEATURES, dtype=torch.float32, device="cuda")
        check(_lib.nnc_features(self.h, _ptr(out)), "nnc_features")
        torch.cuda.synchronize()
        return out

    def profile_enable(self, on: bool = True) -> None:
        check(_lib.nnc_profile_enable(self.h, 1 if on else 0), "nnc_profile_enable")

    def profile_read(self, reset: bool = True) -> dict:
        """Per kernel class: (total ms, launches) of the timed launches (synchronises)."""
        p = Profile()
        check(_lib.nnc_profile_read(self.h, ctypes.byref(p), 1 if reset else 0), "nnc_profile_read")
        return {name: (p.ms[k], p.count[k]) for k, name in enumerate(KERNEL_CLASSES)}

    def snapshot(self, into: Snapshot | None = None) -> Snapshot:
        if into is not None:
            check(_lib.nnc_snapshot_update(self.h, into.handle), "nnc_snapshot_update")
            return into
        h = ctypes.c_void_p()
        check(_lib.nnc_snapshot(self.h, ctypes.byref(h)), "nnc_snapshot")
        return Snapshot(h.value)

    def restore(self, snap: Snapshot) -> None:
        check(_lib.nnc_restore(self.h, snap.handle), "nnc_restore")


class BatchSnapshot:
    def __init__(self, handle: int):
        self.handle = handle

    def __del__(self):
        if self.handle and _lib is not None:
            _lib.nnc_batch_snap_free(self.handle)
            self.handle = 0


class NNCBatch:
    """Many independent scenes advanced together (one launch per kernel for all scenes).

    Positions are one concatenated float32 CUDA tensor: scene s occupies the
    [d_s, n_s] block starting at ``coord_off[s]``."""

    def __init__(self, ns, ds, grids=None, lanes: int = 0, guard: float = -1.0, refresh: float = 0.0,
                 stream: int | None = None, features: bool = False, eager: bool = False, timing: bool = False,
                 budget: bool = False):
        """lanes: lanes per query (1, 4, 8, 16, 32 or 64; 4 serves plane scenes only, cube
        scenes then use 16; 0 = 4 in the plane and 8 in the cube);
        eager: launch each step's kernels directly instead of through the library's graph;
        timing: per-scene wall-clock cost accounting (stats' t_filter_us, t_grid_us, t_query_us);
        budget: the per-point motion budget in every scene (NNC_BATCH_BUDGET)."""
        import numpy as np
        lib = load()
        self.S = len(ns)
        self._n = np.ascontiguousarray(ns, dtype=np.int64)
        self._d = np.ascontiguousarray(ds, dtype=np.int32)
        self._g = None if grids is None else np.ascontiguousarray(grids, dtype=np.int32)
        self.stream = _stream() if stream is None else stream
        cfg = BatchConfig(scenes=self.S, n=self._n.ctypes.data, d=self._d.ctypes.data,
                          grid_g=0 if self._g is None else self._g.ctypes.data, lanes=int(lanes),
                          guard=float(guard), refresh=float(refresh), stream=self.stream,
                          flags=(1 if features else 0) | (2 if eager else 0) | (4 if timing else 0)
                          | (8 if budget else 0))
        h = ctypes.c_void_p()
        check(lib.nnc_batch_create(ctypes.byref(h), ctypes.byref(cfg)), "nnc_batch_create")
        self.h = h.value
        self.point_off = np.zeros(self.S + 1, np.int64)
        self.coord_off = np.zeros(self.S + 1, np.int64)
        check(lib.nnc_batch_offsets(self.h, self.point_off.ctypes.data, self.coord_off.ctypes.data),
              "nnc_batch_offsets")
        self._keep = []

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.nnc_batch_destroy(self.h)
        self.h = None

    def __del__(self):
        self.close()

    def init(self, pos: torch.Tensor) -> None:
        self._keep = [pos]
        check(_lib.nnc_batch_init(self.h, _ptr(pos)), "nnc_batch_init")

    def step(self, pos: torch.Tensor, policy: int = POLICY_REPAIR, tau: float = 0.5) -> None:
        self._keep = (self._keep + [pos])[-2:]
        check(_lib.nnc_batch_step(self.h, _ptr(pos), int(policy), float(tau)), "nnc_batch_step")

    def snapshot(self, into=None):
        """A device copy of the whole batch state (BatchSnapshot; into: overwrite that one)."""
        if into is not None:
            check(_lib.nnc_batch_snapshot_update(self.h, into.handle), "nnc_batch_snapshot_update")
            return into
        h = ctypes.c_void_p()
        check(_lib.nnc_batch_snapshot(self.h, ctypes.byref(h)), "nnc_batch_snapshot")
        return BatchSnapshot(h.value)

    def restore(self, snap) -> None:
        check(_lib.nnc_batch_restore(self.h, snap.handle), "nnc_batch_restore")

    def selector_load(self, params: torch.Tensor) -> None:
        if params.numel() != SELECTOR_PARAMS or params.dtype != torch.float32:
            raise ValueError("selector parameters: float32 tensor of 4738 values")
        check(_lib.nnc_batch_selector_load(self.h, _ptr(params)), "nnc_batch_selector_load")

    def selector_band(self, lo: float, hi: float) -> None:
        """Candidate fractions [lo, hi) in which the learned policy asks the network."""
        check(_lib.nnc_batch_selector_band(self.h, float(lo), float(hi)), "nnc_batch_selector_band")

    def stats(self) -> list:
        arr = (SceneStats * self.S)()
        check(_lib.nnc_batch_scene_stats(self.h, arr), "nnc_batch_scene_stats")
        out = []
        for st in arr:
            d = {k: getattr(st, k) for k, _ in SceneStats._fields_ if k != "features"}
            d["features"] = list(st.features)
            out.append(d)
        return out

    def state(self) -> dict:
        st = State()
        check(_lib.nnc_batch_get_state(self.h, ctypes.byref(st)), "nnc_batch_get_state")
        n = int(st.n)
        spec = [("nn", torch.int32, 4), ("d1", torch.float32, 4), ("d2", torch.float32, 4),
                ("e", torch.float64, 8), ("cell", torch.int32, 4), ("fail", torch.uint8, 1)]
        out = {}
        for name, dt, sz in spec:
            t = torch.empty(n, dtype=dt, device="cuda")
            out[name] = copy_from_device(t, getattr(st, name), n * sz, self.stream)
        torch.cuda.synchronize()
        return out


# ---- selector network kernels ---------------------------------------------------------

def mlp_grad(params: torch.Tensor, X: torch.Tensor, y: torch.Tensor, w: torch.Tensor,
             workspace: torch.Tensor | None = None):
    """(loss, grad) of the weighted cross-entropy on a batch, by the HIP kernels."""
    B = X.shape[0]
    nbytes = load().nnc_mlp_workspace_bytes(B)
    if workspace is None or workspace.numel() * workspace.element_size() < nbytes:
        workspace = torch.empty(max(1, nbytes // 4), dtype=torch.float32, device=X.device)
    g = torch.empty(SELECTOR_PARAMS, dtype=torch.float32, device=X.device)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    check(_lib.nnc_mlp_grad(_ptr(params), _ptr(X), _ptr(y), _ptr(w), B, _ptr(workspace), _ptr(g), _ptr(loss),
                            _stream()), "nnc_mlp_grad")
    return loss, g


MLP_STATIC_MAX_B = 4096


def mlp_grad_static(params: torch.Tensor, X: torch.Tensor, y: torch.Tensor, w: torch.Tensor):
    """(loss, grad) like mlp_grad, through the entry point that allocates nothing
    (its workspace is the library's fixed per-device array; B <= MLP_STATIC_MAX_B)."""
    B = X.shape[0]
    g = torch.empty(SELECTOR_PARAMS, dtype=torch.float32, device=X.device)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    check(load().nnc_mlp_grad_static(_ptr(params), _ptr(X), _ptr(y), _ptr(w), B, _ptr(g), _ptr(loss), _stream()),
          "nnc_mlp_grad_static")
    return loss, g


def mlp_adam(params, m, v, grad, step: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8) -> None:
    check(_lib.nnc_mlp_adam(_ptr(params), _ptr(m), _ptr(v), _ptr(grad), int(step), float(lr), float(beta1),
                            float(beta2), float(eps), _stream()), "nnc_mlp_adam")


def mlp_forward(params: torch.Tensor, X: torch.Tensor) -> torch.Tensor:
    logits = torch.empty((X.shape[0], 2), dtype=torch.float32, device=X.device)
    check(load().nnc_mlp_forward(_ptr(params), _ptr(X), X.shape[0], _ptr(logits), _stream()), "nnc_mlp_forward")
    return logits
