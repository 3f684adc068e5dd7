"""CPU oracle of the certificate-maintenance state machine: TEST INFRASTRUCTURE ONLY.

Only the tests, the package's smoke check and the benchmark's CPU-baseline leg
may import this module.  It shares no code with the GPU path; the one thing the
two sides have in common is the seeded input generator (``synth``).

The method (Section 2, Definition 1, Lemma 1, Definition 2, Algorithm 1 and the
appendix's cumulative clock), written out in plain NumPy plus one brute-force C
routine for the certificates themselves:

* certificate of point i: (nn_i, d1_i, d2_i), by brute force over all points
  (``nncert_oracle.c`` states the exact binary32 arithmetic);
* clearance c_i = d2_i - d1_i (binary32 subtraction), validity radius c_i / 4;
* per step, eps_t = the largest displacement of any point (Algorithm 1, its
  first statement), measured as sqrtf of the largest binary32 squared
  displacement;
* clock S_t = S_{t-1} + eps_t in binary64 (appendix, per-step cost section:
  the sum of per-step maxima);
* a certificate last recomputed at clock S_i stays valid while
  S_t - S_i < c_i / 4 (the appendix applies Theorem 2 to the accumulated
  displacement); the point is a repair candidate once S_t reaches its expiry
  key e_i = S_i + c_i / 4.  A guard gamma widens the candidate set to absorb
  binary32 rounding:  e_i = S_i + (c_i - gamma * d2_i) * K,  K = 1 / (4 + 4 gamma),
  all in binary64;  gamma = 0 is the paper's key exactly;
* candidates are re-certified (repair) or every point is (rebuild); a
  certificate fails when its nearest neighbour changes (Definition 2);
* every point's grid cell is brought up to date every step (Algorithm 1);
  cell of x: per axis g = clamp(floor(fl32(x * G)), 0, G-1), id = gx + G*(gy + G*gz);
* normalised repair-frontier entropy (Definition 2) over the current cells:
  H = (ln|F| - sum_k n_k ln n_k / |F|) / ln C, with C the number of occupied
  cells; H = 0 when F is empty or C <= 1.

The literal reading of Algorithm 1 across many steps (a point is a candidate
when its possibly stale clearance is at most 4 * eps_t of this step alone) is
kept as ``rule="literal"`` so that a test can show it misses failures.

``rule="budget"`` is the tighter per-point safe set the Limitations section
asks for (a per-point motion budget in place of the global step bound): a
point whose key has expired is re-tested against its kept certificate
(nn = j, d2, made at clock S_i).  Every point has moved at most
D = S_t - S_i since, so every k != j is at least d2 - 2 D from i now, while j
is at its current distance r = |p_i - p_j| (binary32 formula, sqrtf).  If
r < d2 - 2 D, j is still the strict nearest neighbour: the certificate is
kept and its key is moved to S_t + (d2 - 2 D - r) / 4 (the gap closes by at
most 4 per unit of clock: r grows by 2 and d2 - 2 D falls by 2); otherwise
the point is a candidate.  With the guard g: the test uses
thr = d2 (1 - g) - 2 (D (1 + g)), gap = thr - r, kept iff gap > 0, new key
S_t + gap * K; all in binary64 in that order.

Before that test the budget rule applies the block-local half of the budget:
every step, the cells a moving point leaves and enters are stamped with the step
number (last_move).  An expired point i whose 3^d block of cells (around its
current cell) holds no stamp later than the step of i's certificate has not moved,
nor has any point that was inside the block; a point outside the block is at least
B - fuzz from i (B: distance from p_i to the outside of the block; fuzz: the cell
boundaries' rounding allowance) and has moved at most D since, so if
(d2 + D)(1 + 2^-20) + fuzz < B no point can have come within d2 of i: the
certificate is still exact, the point is not a candidate and its key becomes
the smallest binary64 value above S_t (it is tested again at the next step in
which anything moves).  Motion confined to one region therefore only makes
candidates of points near that region.
"""
from __future__ import annotations

import ctypes
import itertools
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nncert_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GUARD_DEFAULT = 2.0 ** -18

FAILED = 0
CANDIDATES = 1


def build(force: bool = False) -> str:
    """Compile the C part of the oracle with gcc (no fused multiply-add)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-fopenmp", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        f32p = ctypes.POINTER(ctypes.c_float)
        f64p = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        _lib.orc_top2_f32.argtypes = [f32p, ctypes.c_int64, ctypes.c_int, i64p, ctypes.c_int64,
                                      i32p, f32p, f32p]
        _lib.orc_nn_f64.argtypes = [f32p, ctypes.c_int64, ctypes.c_int, i64p, ctypes.c_int64,
                                    i32p, f64p]
        _lib.orc_pair_sqdist64.argtypes = [f32p, ctypes.c_int64, ctypes.c_int, i64p, i64p,
                                           ctypes.c_int64, f64p]
        _lib.orc_threads.restype = ctypes.c_int
        _lib.orc_set_threads.argtypes = [ctypes.c_int]
        _lib.orc_pair_sqdist32.argtypes = [f32p, ctypes.c_int64, ctypes.c_int, i64p, i64p,
                                           ctypes.c_int64, f32p]
    return _lib


def set_threads(k: int) -> None:
    """Thread count of the C part's parallel loops from now on."""
    lib().orc_set_threads(int(k))


def threads() -> int:
    """OpenMP threads used by the brute-force loops."""
    return int(lib().orc_threads())


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _soa(pos: np.ndarray) -> np.ndarray:
    pos = np.ascontiguousarray(pos, dtype=np.float32)
    if pos.ndim != 2 or pos.shape[0] not in (2, 3):
        raise ValueError("positions must be float32 [d][n] with d in {2, 3}")
    return pos


# --- certificates by brute force (Definition 1) -------------------------------------

def top2(pos: np.ndarray, queries=None):
    """(nn int32, d1 float32, d2 float32) of the queried points (default: all)."""
    pos = _soa(pos)
    d, n = pos.shape
    q = np.arange(n, dtype=np.int64) if queries is None else np.ascontiguousarray(queries, np.int64)
    nn = np.empty(q.size, np.int32)
    d1 = np.empty(q.size, np.float32)
    d2 = np.empty(q.size, np.float32)
    if q.size:
        lib().orc_top2_f32(_ptr(pos, ctypes.c_float), n, d, _ptr(q, ctypes.c_int64), q.size,
                           _ptr(nn, ctypes.c_int32), _ptr(d1, ctypes.c_float), _ptr(d2, ctypes.c_float))
    return nn, d1, d2


def nn_f64(pos: np.ndarray, queries=None):
    """Nearest neighbour under binary64 distances of the binary32 coordinates."""
    pos = _soa(pos)
    d, n = pos.shape
    q = np.arange(n, dtype=np.int64) if queries is None else np.ascontiguousarray(queries, np.int64)
    nn = np.empty(q.size, np.int32)
    s = np.empty(q.size, np.float64)
    if q.size:
        lib().orc_nn_f64(_ptr(pos, ctypes.c_float), n, d, _ptr(q, ctypes.c_int64), q.size,
                         _ptr(nn, ctypes.c_int32), _ptr(s, ctypes.c_double))
    return nn, s


def pair_sqdist64(pos, a, b):
    """Binary64 squared distance of the listed pairs (a[k], b[k]) of binary32 points
    (the distance of the tie audit: exact up to binary64 rounding)."""
    pos = _soa(pos)
    d, n = pos.shape
    a = np.ascontiguousarray(a, np.int64)
    b = np.ascontiguousarray(b, np.int64)
    out = np.empty(a.size, np.float64)
    if a.size:
        lib().orc_pair_sqdist64(_ptr(pos, ctypes.c_float), n, d, _ptr(a, ctypes.c_int64),
                                _ptr(b, ctypes.c_int64), a.size, _ptr(out, ctypes.c_double))
    return out


def pair_sqdist32(pos, a, b):
    pos = _soa(pos)
    d, n = pos.shape
    a = np.ascontiguousarray(a, np.int64)
    b = np.ascontiguousarray(b, np.int64)
    out = np.empty(a.size, np.float32)
    if a.size:
        lib().orc_pair_sqdist32(_ptr(pos, ctypes.c_float), n, d, _ptr(a, ctypes.c_int64),
                                _ptr(b, ctypes.c_int64), a.size, _ptr(out, ctypes.c_float))
    return out


# --- the pieces of Algorithm 1 ------------------------------------------------------

def cells(pos: np.ndarray, G: int, lo=None, hi=None) -> np.ndarray:
    """Linear cell id of every point: x fastest, then y, then z (Algorithm 1's index order).

    The grid covers [0,1]^d, or the box [lo, hi) when given: per axis
    floor(fl32(fl32(x - lo) * s)), s = fl32(G / (hi - lo)) with the division in binary64."""
    pos = _soa(pos)
    if not np.all(np.isfinite(pos)):
        raise FloatingPointError("non-finite coordinate")
    if lo is None:
        q = pos * np.float32(G)                   # binary32 product
    else:
        d = pos.shape[0]
        lo32 = np.asarray(lo, np.float32)[:d, None]
        hi32 = np.asarray(hi, np.float32)[:d, None]
        s = (np.float64(G) / (hi32.astype(np.float64) - lo32.astype(np.float64))).astype(np.float32)
        q = (pos - lo32) * s                      # two binary32 roundings
    g = np.clip(np.floor(q), 0, G - 1).astype(np.int64)
    cid = g[-1].copy()
    for k in range(pos.shape[0] - 2, -1, -1):     # id = g0 + G*(g1 + G*g2)
        cid = g[k] + G * cid
    return cid.astype(np.int32)


def max_step(p_old: np.ndarray, p_new: np.ndarray) -> np.float32:
    """eps_t: sqrtf of the largest binary32 squared displacement (0 for no points)."""
    p_old = _soa(p_old)
    p_new = _soa(p_new)
    if p_old.shape[1] == 0:
        return np.float32(0.0)
    dx = p_new[0] - p_old[0]
    s = dx * dx
    for k in range(1, p_old.shape[0]):
        dk = p_new[k] - p_old[k]
        s = s + dk * dk
    return np.sqrt(np.max(s))


def clearance(d1: np.ndarray, d2: np.ndarray) -> np.ndarray:
    """c = d2 - d1 in binary32 (Definition 1); +inf when d2 is +inf."""
    with np.errstate(invalid="ignore"):
        c = (d2 - d1).astype(np.float32)
    return np.where(np.isinf(d2), np.float32(np.inf), c)


def expiry_key(S_i: float, d1: np.ndarray, d2: np.ndarray, guard: float) -> np.ndarray:
    """Clock value at which a certificate computed at clock S_i must be revisited."""
    K = 1.0 / (4.0 + 4.0 * guard)
    c = clearance(d1, d2).astype(np.float64)
    with np.errstate(invalid="ignore"):
        num = c - guard * d2.astype(np.float64)
        e = np.float64(S_i) + num * K
    return np.where(np.isinf(d2), np.inf, e)


def entropy(members: np.ndarray, cell: np.ndarray):
    """(H, m, C, |F|) of the set ``members`` (bool mask over points) by current cell."""
    occupied = np.unique(cell)
    C = int(occupied.size)
    fc = cell[members]
    F = int(fc.size)
    if F == 0:
        return 0.0, 0, C, 0
    _, counts = np.unique(fc, return_counts=True)
    m = int(counts.size)
    if C <= 1:
        return 0.0, m, C, F
    nk = counts.astype(np.float64)
    H = (math.log(F) - float(np.sum(nk * np.log(nk))) / F) / math.log(C)
    return H, m, C, F


def gyration(pos: np.ndarray, members: np.ndarray):
    """Radius of gyration sqrt(mean |p_i - c|^2) of the member points (boolean mask or
    indices) about their centroid c, and c (z = 0 in the plane), in binary64 by the
    plain two-pass definition: the dataset's spatial-spread descriptor of a frontier
    (Section 6 names it; its definition is this reading).  (0, 0) for no members."""
    pos = _soa(pos).astype(np.float64)
    idx = np.flatnonzero(members) if np.asarray(members).dtype == bool else np.asarray(members, np.int64)
    cen = np.zeros(3)
    if idx.size == 0:
        return 0.0, cen
    P = np.zeros((3, idx.size))
    P[:pos.shape[0]] = pos[:, idx]
    cen = P.mean(axis=1)
    return float(np.sqrt(np.mean(np.sum((P - cen[:, None]) ** 2, axis=0)))), cen


@dataclass
class StepResult:
    eps: np.float32
    S: float
    candidates: np.ndarray  # int64, ascending


@dataclass
class OracleScene:
    """One moving point set and its certificates (the state of Algorithm 1)."""
    d: int
    n: int
    G: int
    guard: float = GUARD_DEFAULT
    rule: str = "clock"             # "clock" (appendix) or "literal" (Algorithm 1 alone)
    lo: tuple = None                # domain box of the grid (None: the unit box)
    hi: tuple = None
    pos: np.ndarray = None
    nn: np.ndarray = None
    d1: np.ndarray = None
    d2: np.ndarray = None
    e: np.ndarray = None
    cell: np.ndarray = None
    fail: np.ndarray = None
    S: float = 0.0
    Si: np.ndarray = None             # clock at which each certificate was computed
    stamp: np.ndarray = None          # step at which each certificate was computed
    last_move: np.ndarray = None      # per cell: last step a moving point left or entered it
    t: int = 0
    pending: StepResult = None
    last_eps: np.float32 = field(default_factory=lambda: np.float32(0))

    def _recompute(self, idx: np.ndarray):
        nn, d1, d2 = top2(self.pos, idx)
        old = self.nn[idx].copy()
        self.nn[idx] = nn
        self.d1[idx] = d1
        self.d2[idx] = d2
        self.e[idx] = expiry_key(self.S, d1, d2, self.guard)
        self.Si[idx] = self.S
        self.stamp[idx] = self.t
        self.fail[:] = False
        self.fail[idx] = nn != old

    def init_certificates(self, pos: np.ndarray):
        self.pos = _soa(pos).copy()
        n = self.n
        self.nn = np.full(n, -1, np.int32)
        self.d1 = np.full(n, np.inf, np.float32)
        self.d2 = np.full(n, np.inf, np.float32)
        self.e = np.full(n, np.inf, np.float64)
        self.Si = np.zeros(n, np.float64)
        self.stamp = np.zeros(n, np.int64)
        self.last_move = np.zeros(self.G ** self.d, np.int64)
        self.t = 0
        self.fail = np.zeros(n, bool)
        self.S = 0.0
        self.cell = cells(self.pos, self.G, self.lo, self.hi)
        self._recompute(np.arange(n, dtype=np.int64))
        self.fail[:] = False
        self.pending = None

    def step(self, pos_new: np.ndarray) -> StepResult:
        pos_new = _soa(pos_new)
        eps = max_step(self.pos, pos_new)
        self.t += 1
        old_cell = self.cell
        self.cell = cells(pos_new, self.G, self.lo, self.hi)  # every cell current (Algorithm 1)
        moved = np.any(pos_new != self.pos, axis=0)
        self.last_move[old_cell[moved]] = self.t
        self.last_move[self.cell[moved]] = self.t
        self.pos_prev = self.pos
        self.pos = pos_new.copy()
        self.S_prev = self.S
        self.S = float(np.float64(self.S) + np.float64(eps))
        self.last_eps = eps
        if self.rule == "clock":
            cand = np.flatnonzero(self.S >= self.e)
        elif self.rule == "budget":
            cand = self._budget_test(np.flatnonzero(self.S >= self.e))
        elif self.rule == "literal":
            c = clearance(self.d1, self.d2).astype(np.float64)
            cand = np.flatnonzero(c <= 4.0 * np.float64(eps))
        else:
            raise ValueError(self.rule)
        self.pending = StepResult(eps, self.S, cand.astype(np.int64))
        return self.pending

    def _budget_test(self, expired: np.ndarray) -> np.ndarray:
        """The per-point budget test of the expired points (module docstring); moves
        the keys of those whose kept neighbour is provably still nearest and returns
        the others, the candidates."""
        if expired.size == 0:
            return expired
        still = self._block_still(expired)
        self.e[expired[still]] = np.nextafter(np.float64(self.S), np.inf)
        expired = expired[~still]
        if expired.size == 0:
            return expired
        g = self.guard
        j = self.nn[expired].astype(np.int64)
        r = np.sqrt(pair_sqdist32(self.pos, expired, j))                 # binary32
        D = np.float64(self.S) - self.Si[expired]
        thr = self.d2[expired].astype(np.float64) * (1.0 - g) - 2.0 * (D * (1.0 + g))
        gap = thr - r.astype(np.float64)
        keep = gap > 0.0
        K = np.float64(1.0) / (np.float64(4.0) + np.float64(4.0) * np.float64(g))
        self.e[expired[keep]] = np.float64(self.S) + gap[keep] * K
        return expired[~keep]

    def _block_still(self, idx: np.ndarray) -> np.ndarray:
        """The block-local test (module docstring) of the points idx: True where no
        cell of the point's 3^d block was stamped after its certificate and no point
        from outside the block can have come within d2."""
        d, G = self.d, self.G
        gid = self.cell[idx].astype(np.int64)
        gc = []
        for _ in range(d):                          # per-axis cell coordinates, x first
            gc.append(gid % G)
            gid = gid // G
        quiet = np.ones(idx.size, bool)
        for offs in itertools.product((-1, 0, 1), repeat=d):
            nb = np.zeros(idx.size, np.int64)
            inside = np.ones(idx.size, bool)
            for k in range(d - 1, -1, -1):
                gk = gc[k] + offs[k]
                inside &= (gk >= 0) & (gk < G)
                nb = nb * G + np.clip(gk, 0, G - 1)
            quiet &= ~inside | (self.last_move[nb] <= self.stamp[idx])
        # distance from p_i to the outside of its block (sides at the grid edge open)
        lo = np.zeros(3) if self.lo is None else np.asarray(self.lo, np.float32).astype(np.float64)
        hi = np.ones(3) if self.hi is None else np.asarray(self.hi, np.float32).astype(np.float64)
        B = np.full(idx.size, np.inf)
        for k in range(d):
            w = (hi[k] - lo[k]) / np.float64(G)
            x = self.pos[k, idx].astype(np.float64)
            low_side = gc[k] - 1 > 0
            B = np.where(low_side, np.minimum(B, x - (lo[k] + (gc[k] - 1).astype(np.float64) * w)), B)
            high_side = gc[k] + 1 < G - 1
            B = np.where(high_side, np.minimum(B, (lo[k] + (gc[k] + 2).astype(np.float64) * w) - x), B)
        mag = 1.0 if self.lo is None else max(1.0, *np.abs(lo[:d]), *np.abs(hi[:d]))
        fuzz = 2.0 ** -20 * mag
        D = np.float64(self.S) - self.Si[idx]
        need = (self.d2[idx].astype(np.float64) + D) * (1.0 + 2.0 ** -20) + fuzz
        return quiet & (need < B)

    def rho_flags(self) -> np.ndarray:
        """The local predictor the paper reports beside the safety rule (Section 4,
        Table 1) for the pending step: rho_i = delta_i / c_i > 1/2, with c_i the kept
        certificate's binary32 clearance and delta_i the step's motion of i plus that of
        its kept nearest neighbour (the paper leaves delta_i undefined; this is the
        reading), each motion sqrt of the binary32 squared displacement (the formula of
        eps_t), summed in binary32; flagged iff 2 delta_i > c_i."""
        if self.pending is None:
            raise RuntimeError("rho without a pending step")
        p0, p1 = self.pos_prev, self.pos
        dx = p1[0] - p0[0]
        s = dx * dx
        for k in range(1, p0.shape[0]):
            dk = p1[k] - p0[k]
            s = s + dk * dk
        move = np.sqrt(s)                      # binary32, correctly rounded
        j = self.nn
        ok = (j >= 0) & (j < self.n)
        delta = move + move[np.where(ok, j, 0)]
        c = clearance(self.d1, self.d2)
        with np.errstate(invalid="ignore"):
            flag = (np.float32(2.0) * delta) > c
        return ok & flag

    def features(self) -> np.ndarray:
        """The six repair-strategy selector inputs of the pending step, as the library
        defines them (Section 3 labels a transition by its fastest strategy; the
        selector predicts that label from these descriptors of the candidate set):
        |F|/N; H of the candidates (Definition 2); ln N; d; m_cand / G^d, the fraction
        of all cells the candidates meet; and eps_t over the median remaining motion
        budget r_i = e_i - S_{t-1} of the certificates of points 0 .. min(N, 1024) - 1
        (a fixed sample) with 0 < r_i < inf, the median
        read from a 64-bin histogram of r by binary exponent (bin = ilogb(r) + 48,
        clamped to [0, 63]; the first bin whose running count reaches half of all,
        represented by 1.5 * 2^(bin - 48)); 0 when no certificate has a finite budget.
        Returned in binary64; the library rounds each to binary32."""
        if self.pending is None:
            raise RuntimeError("features without a pending step")
        n = self.n
        cand = self.pending.candidates
        H, m, C, F = self.frontier_entropy(CANDIDATES, cand)
        r = self.e[:1024] - self.S_prev
        r = r[(r > 0) & np.isfinite(r)]
        h = np.zeros(64, np.int64)
        if r.size:
            ex = np.frexp(r)[1] - 1          # ilogb of a positive finite binary64
            np.add.at(h, np.clip(ex + 48, 0, 63), 1)
        V = int(h.sum())
        radius = 0.0
        if V:
            b = int(np.argmax(2 * np.cumsum(h) >= V))
            radius = 1.5 * 2.0 ** (b - 48)
        return np.array([F / n if n else 0.0, H, math.log(n) if n else 0.0, self.d,
                         m / float(self.G) ** self.d,
                         float(self.pending.eps) / radius if radius > 0 else 0.0])

    def repair(self, frontier=None):
        if self.pending is None:
            raise RuntimeError("repair without a pending step")
        idx = self.pending.candidates if frontier is None else np.ascontiguousarray(frontier, np.int64)
        self._recompute(idx)
        self.pending = None

    def rebuild(self):
        if self.pending is None:
            raise RuntimeError("rebuild without a pending step")
        self._recompute(np.arange(self.n, dtype=np.int64))
        self.pending = None

    def frontier_entropy(self, which: int = FAILED, candidates=None):
        if which == FAILED:
            mask = self.fail
        else:
            mask = np.zeros(self.n, bool)
            mask[candidates] = True
        return entropy(mask, self.cell)

    def audit(self):
        """Points whose kept nearest neighbour differs from brute force now (misses)."""
        nn_bf, _, _ = top2(self.pos)
        return np.flatnonzero(nn_bf != self.nn)
