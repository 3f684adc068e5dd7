"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: the binary32 formula is checked
against an exact rational emulation, the real-number certificate against exact
brute force, the state machine against hand-derived constructions from the
appendix, closed forms of the entropy, invariants that hold at any size, and
special cases whose answer is known without computing it.
"""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import exact, model

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U = 2.0 ** -24


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# --- binary32 arithmetic of the certificate -----------------------------------------

def test_round_f32_agrees_with_hardware_conversion():
    g = np.random.default_rng(7)
    vals = np.concatenate([g.standard_normal(2000) * 10.0 ** g.integers(-40, 30, 2000),
                           [1e-45, 3e-39, 1.17549435e-38, 0.5, 1.0, 3.4e38]])
    for v in vals:
        assert exact.round_f32(Fraction(float(v))) == Fraction(float(np.float32(v)))


def test_sqrt_f32_agrees_with_hardware_sqrt():
    g = np.random.default_rng(8)
    vals = np.abs(g.standard_normal(3000).astype(np.float32)) * np.float32(2.0) ** g.integers(-60, 60, 3000)
    for v in vals.astype(np.float32):
        assert exact.sqrt_f32(exact.exact(v)) == exact.exact(np.sqrt(v))


def _random_scene(g, n, d, kind):
    if kind == "uniform":
        p = g.random((d, n))
    elif kind == "lattice":        # exact ties everywhere
        p = g.integers(0, 4, (d, n)) / 8.0
    elif kind == "tiny":           # distances near the subnormal range
        p = 0.5 + g.standard_normal((d, n)) * 1e-19
    elif kind == "duplicates":
        p = g.random((d, n))
        p[:, n // 2:] = p[:, : n - n // 2]
    else:
        p = g.standard_normal((d, n)) * 100.0
    return np.ascontiguousarray(p, dtype=np.float32)


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("kind", ["uniform", "lattice", "tiny", "duplicates", "wide"])
def test_c_certificate_is_the_binary32_formula_bit_for_bit(d, kind):
    g = np.random.default_rng(100 + d * 10 + len(kind))
    for n in (1, 2, 3, 17, 33):
        pos = _random_scene(g, n, d, kind)
        nn, d1, d2 = model.top2(pos)
        P = exact.coords(pos)
        for i in range(n):
            enn, ed1, ed2 = exact.top2_f32(P, i)
            assert nn[i] == enn
            assert (d1[i] == np.inf) if ed1 is None else exact.exact(d1[i]) == ed1
            assert (d2[i] == np.inf) if ed2 is None else exact.exact(d2[i]) == ed2


@pytest.mark.parametrize("d", [2, 3])
def test_binary32_nn_is_the_real_nn_up_to_rounding(d):
    """Where binary32 picks another neighbour than exact arithmetic, it is a near-tie."""
    g = np.random.default_rng(200 + d)
    for _ in range(6):
        pos = _random_scene(g, 40, d, "uniform")
        nn, d1, d2 = model.top2(pos)
        P = exact.coords(pos)
        for i in range(pos.shape[1]):
            rnn, S1, S2 = exact.top2_real(P, i)
            if nn[i] != rnn:
                s_other = exact.sqdist_real(P, i, int(nn[i]))
                assert abs(s_other - S1) <= Fraction(16) * Fraction(U) * S1
            # d1, d2 within a few units in the last place of the exact distances
            for dv, Sv in ((d1[i], S1), (d2[i], S2)):
                assert abs(exact.exact(dv) ** 2 - Sv) <= Fraction(8) * Fraction(U) * Sv


def test_distance_is_symmetric():
    g = np.random.default_rng(3)
    pos = _random_scene(g, 500, 3, "wide")
    a = g.integers(0, 500, 5000)
    b = g.integers(0, 500, 5000)
    assert np.array_equal(model.pair_sqdist32(pos, a, b).view(np.uint32),
                          model.pair_sqdist32(pos, b, a).view(np.uint32))


def test_binary64_audit_routine_is_exact_brute_force():
    g = np.random.default_rng(4)
    pos = _random_scene(g, 30, 3, "uniform")
    nn64, s64 = model.nn_f64(pos)
    P = exact.coords(pos)
    for i in range(30):
        rnn, S1, _ = exact.top2_real(P, i)
        assert nn64[i] == rnn
        assert abs(Fraction(float(s64[i])) - S1) <= Fraction(4) * Fraction(2.0 ** -53) * S1


# --- the pieces of the step ---------------------------------------------------------

def test_cell_formula_against_exact_arithmetic():
    G = 15
    vals = [0.0, -0.0, 1.0, -1e-30, -3.0, 1.0000001, 7.0, 2.0 ** -149]
    vals += [k / G for k in range(G + 1)]
    vals += list(np.nextafter(np.float32([k / G for k in range(1, G)]), np.float32(0)))
    vals += list(np.nextafter(np.float32([k / G for k in range(1, G)]), np.float32(2)))
    xs = np.array(vals, dtype=np.float32)
    pos = np.stack([xs, xs[::-1].copy()])
    got = model.cells(pos, G)
    for j in range(xs.size):
        want = 0
        for k in (1, 0):
            q = exact.round_f32(exact.exact(pos[k, j]) * G)
            g = min(max(math.floor(q), 0), G - 1)
            want = g + G * want
        assert got[j] == want


def test_cell_rejects_nan():
    with pytest.raises(FloatingPointError):
        model.cells(np.array([[0.5, np.nan], [0.1, 0.2]], np.float32), 4)


def test_max_step_is_sqrt_of_the_largest_binary32_squared_displacement():
    g = np.random.default_rng(5)
    for d in (2, 3):
        a = _random_scene(g, 25, d, "uniform")
        b = (a + g.standard_normal(a.shape).astype(np.float32) * np.float32(1e-3)).astype(np.float32)
        eps = model.max_step(a, b)
        A, B = exact.coords(a), exact.coords(b)
        best = Fraction(0)
        for j in range(25):
            s = None
            for k in range(d):
                dk = exact.round_f32(B[k][j] - A[k][j])
                sq = exact.round_f32(dk * dk)
                s = sq if s is None else exact.round_f32(s + sq)
            best = max(best, s)
        assert exact.exact(eps) == exact.sqrt_f32(best)


def test_expiry_key_is_the_guarded_validity_radius():
    g = np.random.default_rng(6)
    d1 = np.abs(g.standard_normal(200)).astype(np.float32)
    d2 = (d1 + np.abs(g.standard_normal(200)).astype(np.float32)).astype(np.float32)
    for guard in (0.0, model.GUARD_DEFAULT):
        S = 0.125
        e = model.expiry_key(S, d1, d2, guard)
        for k in range(200):
            c = exact.round_f32(exact.exact(d2[k]) - exact.exact(d1[k]))
            real = Fraction(S) + (c - Fraction(guard) * exact.exact(d2[k])) / (4 + 4 * Fraction(guard))
            assert abs(Fraction(float(e[k])) - real) <= Fraction(2.0 ** -50) * (abs(real) + 1)
    # no second neighbour: never expires
    assert model.expiry_key(0.0, np.float32([1.0]), np.float32([np.inf]), 0.0)[0] == np.inf


# --- the appendix's tightness construction -----------------------------------------

def _line_scene(eta, order, d1, eps, d):
    """i = point 0 at the origin, a at d1, k at -(d1 + eta*eps), on the x axis."""
    xi, xa, xk = 0.0, d1, -(d1 + eta * eps)
    ia, ik = (1, 2) if order == "a<k" else (2, 1)
    x0 = np.zeros(3)
    x0[0], x0[ia], x0[ik] = xi, xa, xk
    x1 = x0.copy()
    x1[0] -= eps           # i toward k
    x1[ia] += eps          # a away from i
    x1[ik] += eps          # k toward i
    p0 = np.full((d, 3), 0.5)
    p1 = np.full((d, 3), 0.5)
    p0[0] += x0
    p1[0] += x1
    return p0.astype(np.float32), p1.astype(np.float32), ia, ik


@pytest.mark.parametrize("guard", [0.0, model.GUARD_DEFAULT])
@pytest.mark.parametrize("d", [2, 3])
def test_theorem2_tightness_construction(guard, d):
    fx = _golden("thm2_tightness.json")
    for case in fx["cases"]:
        p0, p1, ia, ik = _line_scene(case["eta"], case["order"], fx["d1"], fx["eps"], d)
        sc = model.OracleScene(d=d, n=3, G=4, guard=guard)
        sc.init_certificates(p0)
        assert sc.nn[0] == ia
        c = float(sc.d2[0]) - float(sc.d1[0])
        assert c == case["eta"] * fx["eps"]
        res = sc.step(p1)
        assert float(res.eps) == fx["eps"]
        assert (0 in set(res.candidates.tolist())) == case["candidate"]
        sc.repair()
        assert bool(sc.fail[0]) == case["nn_changes"]
        assert sc.nn[0] == (ik if case["nn_changes"] else ia)
        assert sc.audit().size == 0


# --- exhaustive lattice enumeration ------------------------------------------------

def _lattice_cases_2d():
    sites = [(x, y) for x in (0.0, 0.5, 1.0) for y in (0.0, 0.5, 1.0)]
    moves = [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)]
    for trip in itertools.permutations(sites, 3):
        for mv in itertools.product(moves, repeat=3):
            p0 = np.array(trip, dtype=np.float64).T
            p1 = p0 + np.array(mv, dtype=np.float64).T / 8.0
            yield p0.astype(np.float32), p1.astype(np.float32)


def test_lattice_enumeration_no_missed_failure_and_superset():
    """Every ordered 3-point configuration of a 3x3 lattice (spacing 1/2) under every
    combination of axis moves of length 1/8 (or none): all arithmetic is exact in
    binary32, ties are everywhere, and the filter must still contain every failure."""
    n_cases = n_fail = n_boundary = 0
    for p0, p1 in _lattice_cases_2d():
        sc = model.OracleScene(d=2, n=3, G=2, guard=0.0)
        sc.init_certificates(p0)
        c = (sc.d2 - sc.d1).astype(np.float64)
        nn_before = sc.nn.copy()
        res = sc.step(p1)
        cand = set(res.candidates.tolist())
        nn_after, _, _ = model.top2(p1)
        failed = set(np.flatnonzero(nn_after != nn_before).tolist())
        assert failed <= cand
        sc.repair()
        assert np.array_equal(sc.nn, nn_after)
        n_cases += 1
        n_fail += len(failed)
        n_boundary += int(np.sum(c == 4.0 * float(res.eps)))
    assert n_cases == 504 * 125
    assert n_fail > 1000 and n_boundary > 1000    # the enumeration does reach the boundary


# --- special cases -----------------------------------------------------------------

def test_zero_motion_breaks_nothing():
    tr = synth.plane_1k(steps=1)
    sc = model.OracleScene(d=2, n=1000, G=15)
    sc.init_certificates(tr.frames[0])
    res = sc.step(tr.frames[0])
    assert res.eps == 0 and res.S == 0.0
    c = (sc.d2 - sc.d1).astype(np.float64)
    assert set(res.candidates.tolist()) == set(np.flatnonzero(c <= model.GUARD_DEFAULT * sc.d2).tolist())
    sc.repair()
    assert not sc.fail.any()


def test_rigid_dyadic_translation_breaks_nothing():
    g = np.random.default_rng(9)
    for d in (2, 3):
        p0 = (g.integers(0, 1024, (d, 3000)) / 1024.0).astype(np.float32)
        p1 = p0.copy()
        p1[0] += np.float32(1.0 / 1024.0)         # every difference is preserved exactly
        sc = model.OracleScene(d=d, n=3000, G=8)
        sc.init_certificates(p0)
        sc.step(p1)
        sc.repair()
        assert not sc.fail.any()
        assert sc.audit().size == 0


def test_tiny_scenes():
    for n in (0, 1, 2):
        p = np.random.default_rng(n).random((3, n)).astype(np.float32)
        sc = model.OracleScene(d=3, n=n, G=3)
        sc.init_certificates(p)
        if n == 1:
            assert sc.nn[0] == -1 and np.isinf(sc.d1[0]) and np.isinf(sc.d2[0])
        if n == 2:
            assert list(sc.nn) == [1, 0] and np.all(np.isinf(sc.d2))
        assert np.all(np.isinf(sc.e))
        res = sc.step(p + np.float32(0.01))
        assert res.candidates.size == 0


# --- the whole state machine on the workloads -------------------------------------

def test_plane_1k_every_step_no_miss_and_fail_set_is_the_true_change():
    tr = synth.plane_1k()
    sc = model.OracleScene(d=2, n=1000, G=15)
    sc.init_certificates(tr.frames[0])
    prev_nn = model.top2(tr.frames[0])[0]
    for t in range(1, tr.steps + 1):
        res = sc.step(tr.frames[t])
        sc.repair()
        nn_now = model.top2(tr.frames[t])[0]
        assert np.array_equal(sc.nn, nn_now)                       # no missed failure
        assert set(np.flatnonzero(sc.fail)) == set(np.flatnonzero(nn_now != prev_nn))
        assert set(np.flatnonzero(sc.fail)) <= set(res.candidates.tolist())
        prev_nn = nn_now


@pytest.mark.parametrize("family", synth.FAMILIES)
def test_cube_16k_families_no_miss_reduced(family):
    tr = synth.make_trajectory(family, 3000, 3, 25, 5e-4, 2000 + synth.FAMILIES.index(family))
    sc = model.OracleScene(d=3, n=3000, G=9)
    sc.init_certificates(tr.frames[0])
    for t in range(1, tr.steps + 1):
        sc.step(tr.frames[t])
        if t % 5 == 0:
            sc.rebuild()
        else:
            sc.repair()
        assert sc.audit().size == 0


@pytest.mark.parametrize("family", synth.FAMILIES + synth.EXTRA_FAMILIES)
@pytest.mark.parametrize("d", [2, 3])
def test_family_steps_stay_within_eps(family, d):
    """Every family's binary32 frames move no point farther than eps per step (to
    the binary32 rounding of the coordinates), so eps is a valid declared bound."""
    eps = 2e-3
    tr = synth.make_trajectory(family, 2000, d, 20, eps, 31 + d)
    fr = tr.frames.astype(np.float64)
    step = np.sqrt(((fr[1:] - fr[:-1]) ** 2).sum(axis=1)).max()
    assert step <= eps * (1.0 + 2.0 ** -20) + 2.0 ** -23


@pytest.mark.parametrize("family", synth.EXTRA_FAMILIES)
@pytest.mark.parametrize("d", [2, 3])
def test_extra_families_no_miss_reduced(family, d):
    """The other five families of the paper's list: no missed failure on every step,
    repairs with a rebuild every fifth step."""
    tr = synth.make_trajectory(family, 2500, d, 25, 2e-3, 2100 + synth.EXTRA_FAMILIES.index(family))
    sc = model.OracleScene(d=d, n=2500, G=9 if d == 3 else 30)
    sc.init_certificates(tr.frames[0])
    for t in range(1, tr.steps + 1):
        sc.step(tr.frames[t])
        if t % 5 == 0:
            sc.rebuild()
        else:
            sc.repair()
        assert sc.audit().size == 0


@pytest.mark.parametrize("family", ["uniform_brownian", "adversarial_crossing", "clustered_drift"])
@pytest.mark.parametrize("d", [2, 3])
def test_previous_certificate_bounds_the_new_second_distance(family, d):
    """The search cut-off of the GPU queries: every point has moved at most S_t - S_i
    since its certificate was made at clock S_i (the clock sums the measured maximum
    steps), so its two old neighbours, hence its new second neighbour, lie within
    d2 + 2 (S_t - S_i).  Checked against binary64 brute force at every step of
    repaired trajectories, with S_i both tracked and recovered from the expiry key
    as the kernels do (e - (c - gamma d2) K), within the kernels' relative slack."""
    n = 1500
    tr = synth.make_trajectory(family, n, d, 25, 2e-3, 900 + d)
    sc = model.OracleScene(d=d, n=n, G=8)
    sc.init_certificates(tr.frames[0])
    K = 1.0 / (4.0 + 4.0 * sc.guard)
    Si = np.zeros(n)                     # clock of each point's certificate
    slack = 2.0 ** -16
    for t in range(1, tr.steps + 1):
        d1_old, d2_old, e_old = sc.d1.copy(), sc.d2.copy(), sc.e.copy()
        res = sc.step(tr.frames[t])
        c = (d2_old - d1_old).astype(np.float32).astype(np.float64)
        Si_key = e_old - (c - sc.guard * d2_old.astype(np.float64)) * K
        assert np.allclose(Si_key, Si, rtol=0, atol=1e-12)
        p = tr.frames[t].astype(np.float64)
        dist = np.sqrt(((p[:, :, None] - p[:, None, :]) ** 2).sum(axis=0))
        np.fill_diagonal(dist, np.inf)
        d2_true = np.partition(dist, 1, axis=1)[:, 1]
        bound = (d2_old.astype(np.float64) + 2.0 * (res.S - Si)) * (1.0 + slack)
        assert np.all(d2_true <= bound), f"step {t}"
        sc.repair()
        Si[res.candidates] = res.S


def test_rho_predictor_on_exact_dyadic_scenes():
    """The local predictor rho_i = delta_i / c_i > 1/2 on three collinear points whose
    distances, clearances and motions are dyadic (exact in binary32): p0 = 0,
    p1 = 1/4, p2 = 1 give nn = (1, 0, 1) and c = (3/4, 1/2, 1/4).  The flags are worked
    out by hand, including the strict boundary 2 delta = c (not flagged), a point
    whose own motion is zero but whose neighbour's is not, and N = 2 (d2 = +inf) and
    N = 1 (no neighbour), which are never flagged."""
    def run(p_old, p_new):
        sc = model.OracleScene(d=2, n=p_old.shape[1], G=4)
        sc.init_certificates(np.asarray(p_old, np.float32))
        sc.step(np.asarray(p_new, np.float32))
        return sc.rho_flags()
    p = np.array([[0.0, 0.25, 1.0], [0.0, 0.0, 0.0]])
    # p0 moves 1/8: delta = (1/8, 1/8, 0) + neighbour motion -> 2 delta = (1/4, 1/4, 0)
    q = p.copy(); q[0, 0] += 0.125
    assert run(p, q).tolist() == [False, False, False]
    # p2 moves 1/8 in y: 2 delta_2 = 1/4 = c_2 exactly -> not flagged (strict)
    q = p.copy(); q[1, 2] += 0.125
    assert run(p, q).tolist() == [False, False, False]
    # p2 moves 1/4: 2 delta_2 = 1/2 > 1/4 -> flagged; p0, p1 unmoved and their
    # neighbours (p1, p0) unmoved -> not flagged
    q = p.copy(); q[1, 2] += 0.25
    assert run(p, q).tolist() == [False, False, True]
    # p0 moves 3/16: 2 delta_0 = 3/8 < 3/4; p1's neighbour p0 moved: 2 delta_1 = 3/8 <
    # 1/2; p2's neighbour p1 unmoved -> none; then 5/16: 2 delta_1 = 5/8 > 1/2 -> p1 only
    q = p.copy(); q[0, 0] -= 0.1875
    assert run(p, q).tolist() == [False, False, False]
    q = p.copy(); q[0, 0] -= 0.3125
    assert run(p, q).tolist() == [False, True, False]
    # N = 2: d2 = +inf, c = +inf; N = 1: nn = -1
    assert run(np.array([[0.0, 0.5], [0.0, 0.0]]), np.array([[0.4, 0.1], [0.0, 0.0]])).tolist() == [False, False]
    assert run(np.array([[0.5], [0.5]]), np.array([[0.0], [0.0]])).tolist() == [False]


def test_literal_algorithm_with_stale_certificates_misses_failures():
    """Read step by step with the clearance of possibly stale certificates, the
    filter of Algorithm 1 does miss failures; the appendix's clock does not."""
    tr = synth.plane_1k()
    literal = model.OracleScene(d=2, n=1000, G=15, rule="literal")
    clock = model.OracleScene(d=2, n=1000, G=15)
    literal.init_certificates(tr.frames[0])
    clock.init_certificates(tr.frames[0])
    misses_literal = misses_clock = 0
    for t in range(1, tr.steps + 1):
        for sc in (literal, clock):
            sc.step(tr.frames[t])
            sc.repair()
        misses_literal += literal.audit().size
        misses_clock += clock.audit().size
    assert misses_clock == 0
    assert misses_literal > 100


def test_first_step_literal_equals_clock_without_guard():
    tr = synth.plane_1k(steps=1)
    a = model.OracleScene(d=2, n=1000, G=15, rule="literal", guard=0.0)
    b = model.OracleScene(d=2, n=1000, G=15, rule="clock", guard=0.0)
    a.init_certificates(tr.frames[0])
    b.init_certificates(tr.frames[0])
    ra, rb = a.step(tr.frames[1]), b.step(tr.frames[1])
    assert np.array_equal(ra.candidates, rb.candidates)


# --- entropy -----------------------------------------------------------------------

def test_entropy_closed_forms():
    for case in _golden("entropy_closed_forms.json")["cases"]:
        H, m, C, F = model.entropy(np.array(case["members"], bool), np.array(case["cells"], np.int32))
        assert (m, C, F) == (case["m"], case["C"], case["F"]), case["name"]
        assert abs(H - case["H"]) <= 1e-12, case["name"]


def test_entropy_lower_bounds_touched_cells_theorem4():
    g = np.random.default_rng(11)
    for _ in range(300):
        n = int(g.integers(1, 400))
        cell = g.integers(0, int(g.integers(1, 60)), n).astype(np.int32)
        members = g.random(n) < g.random()
        H, m, C, F = model.entropy(members, cell)
        assert 0.0 <= H <= 1.0 + 1e-12
        if F:
            assert m >= C ** H * (1 - 1e-12)


def test_box_cells_equal_the_cells_of_exactly_normalised_coordinates():
    """A domain box [-1, 3)^d maps by x -> (x + 1) / 4, exact for dyadic coordinates, so
    the box formula must give the unit-box cells of the normalised points; the unit
    box given explicitly is the default formula."""
    g = np.random.default_rng(17)
    for d in (2, 3):
        k = g.integers(-40, 300, (d, 2000))            # some points outside the box
        pos = (k / 64.0 - 1.0).astype(np.float32)
        G = 24
        boxed = model.cells(pos, G, lo=(-1.0,) * 3, hi=(3.0,) * 3)
        unit = model.cells(((pos.astype(np.float64) + 1.0) / 4.0).astype(np.float32), G)
        assert np.array_equal(boxed, unit)
        p01 = g.random((d, 500)).astype(np.float32)
        assert np.array_equal(model.cells(p01, 17, lo=(0.0,) * 3, hi=(1.0,) * 3), model.cells(p01, 17))


# --- the binary64 tie audit and the selector features ------------------------------------

def test_binary64_pair_distance_against_exact_arithmetic():
    """pair_sqdist64 (the distance of the tie audit) is the real squared distance up to
    binary64 rounding, and exact on dyadic coordinates with few bits."""
    g = np.random.default_rng(41)
    for d in (2, 3):
        pos = _random_scene(g, 60, d, "uniform")
        a = g.integers(0, 60, 400)
        b = g.integers(0, 60, 400)
        s = model.pair_sqdist64(pos, a, b)
        P = exact.coords(pos)
        for k in range(400):
            S = exact.sqdist_real(P, int(a[k]), int(b[k]))
            assert abs(Fraction(float(s[k])) - S) <= Fraction(4) * Fraction(2.0 ** -53) * S
        lat = _random_scene(g, 60, d, "lattice")
        s = model.pair_sqdist64(lat, a, b)
        P = exact.coords(lat)
        for k in range(400):
            assert Fraction(float(s[k])) == exact.sqdist_real(P, int(a[k]), int(b[k]))


def _tie_audit(pos):
    """(near_ties, errors) of binary32 brute force against binary64 brute force: where
    the two nearest neighbours differ, a near-tie if their binary64 squared distances
    are within 16u of each other (u = 2^-24), otherwise an error."""
    nn32, _, _ = model.top2(pos)
    nn64, s64 = model.nn_f64(pos)
    diff = np.flatnonzero(nn32 != nn64)
    if diff.size == 0:
        return 0, 0
    s_other = model.pair_sqdist64(pos, diff, nn32[diff])
    near = np.abs(s_other - s64[diff]) <= 16.0 * U * s64[diff]
    return int(near.sum()), int((~near).sum())


def test_binary64_tie_audit_of_the_workloads():
    """Every frame of plane_1k and every 25th frame of the five N = 16000 cube
    trajectories: the binary32 certificates pick the binary64 nearest neighbour except
    at near-ties, never farther than the rounding band."""
    near = err = frames = 0
    tr = synth.plane_1k()
    for f in tr.frames:
        a, b = _tie_audit(f)
        near, err, frames = near + a, err + b, frames + 1
    for fam in synth.FAMILIES:
        tr = synth.cube_16k(fam)
        for t in range(0, tr.steps + 1, 25):
            a, b = _tie_audit(tr.frames[t])
            near, err, frames = near + a, err + b, frames + 1
    print(f"tie audit: {frames} frames, {near} binary32 near-ties, {err} errors")
    assert err == 0


def test_selector_features_median_bin_and_counts():
    """The oracle's selector features of a pending step against their definitions
    recomputed by plain loops: candidate fraction, touched cells over all cells, ln N,
    d, and the budget median: the bin reported holds the element of rank ceil(V/2) of
    the sorted budgets of the first 1024 certificates."""
    tr = synth.make_trajectory("clustered_drift", 3000, 3, 4, 1e-3, 77)
    sc = model.OracleScene(d=3, n=3000, G=12)
    sc.init_certificates(tr.frames[0])
    for t in range(1, 5):
        e_before, S_prev = sc.e.copy(), sc.S
        res = sc.step(tr.frames[t])
        f = sc.features()
        cand = res.candidates
        assert f[0] == cand.size / 3000
        assert len({int(sc.cell[i]) for i in cand}) / 12 ** 3 == f[4]
        assert f[2] == math.log(3000) and f[3] == 3
        r = sorted(float(e_before[i] - S_prev) for i in range(1024)
                   if e_before[i] - S_prev > 0 and math.isfinite(e_before[i] - S_prev))
        med = r[(len(r) + 1) // 2 - 1]
        radius = float(res.eps) / f[5]
        lo = radius / 1.5
        assert lo <= med < 2 * lo, (t, med, radius)
        H, m, C, F = sc.frontier_entropy(model.CANDIDATES, cand)
        assert f[1] == H
        sc.repair()


# --- the per-point motion budget (rule "budget") -------------------------------------------

def _line_scene_moves(eta, order, d1, eps, d, moves):
    p0, p1, ia, ik = _line_scene(eta, order, d1, eps, d)
    if moves == "k":                       # only k moves (toward i); i and a stay
        p1 = p0.copy()
        p1[0, ik] = np.float32(float(p0[0, ik]) + eps)
    return p0, p1, ia, ik


@pytest.mark.parametrize("guard", [0.0, model.GUARD_DEFAULT])
@pytest.mark.parametrize("d", [2, 3])
def test_budget_rule_line_constructions(guard, d):
    """The per-point test on Theorem 2's line: as tight as the clock rule when i and
    its neighbour move apart (the theorem's worst case), strictly tighter when they
    stand still; the key of a kept point moves to S_t + gap/4; never a missed failure."""
    fx = _golden("budget_tightness.json")
    eps = fx["eps"]
    for case in fx["cases"]:
        p0, p1, ia, ik = _line_scene_moves(case["eta"], case["order"], fx["d1"], eps, d, case["moves"])
        for rule in ("budget", "clock"):
            sc = model.OracleScene(d=d, n=3, G=4, guard=guard, rule=rule)
            sc.init_certificates(p0)
            assert sc.nn[0] == ia and float(sc.d2[0]) - float(sc.d1[0]) == case["eta"] * eps
            res = sc.step(p1)
            assert float(res.eps) == eps
            want = case["candidate"] if rule == "budget" else case["clock_candidate"]
            assert (0 in set(res.candidates.tolist())) == want, (case, rule)
            if rule == "budget" and guard == 0.0 and case["key_over_eps"] is not None:
                assert sc.e[0] == case["key_over_eps"] * eps, case
            sc.repair()
            assert bool(sc.fail[0]) == case["nn_changes"]
            assert sc.audit().size == 0


def test_budget_rule_lattice_enumeration_no_miss_and_subset():
    """All 504 x 125 lattice configurations: the per-point rule's candidates are a
    subset of the clock rule's, contain every failure, and the enumeration reaches
    the rule's boundary (|p_i - p_nn| = d2 - 2 eps exactly)."""
    n_cases = n_strict = n_boundary = 0
    for p0, p1 in _lattice_cases_2d():
        a = model.OracleScene(d=2, n=3, G=2, guard=0.0, rule="budget")
        b = model.OracleScene(d=2, n=3, G=2, guard=0.0)
        a.init_certificates(p0)
        b.init_certificates(p0)
        nn_before = a.nn.copy()
        r = np.sqrt(model.pair_sqdist32(p1, np.arange(3), nn_before.astype(np.int64))).astype(np.float64)
        thr = a.d2.astype(np.float64)
        ra, rb = a.step(p1), b.step(p1)
        ca, cb = set(ra.candidates.tolist()), set(rb.candidates.tolist())
        thr = thr - 2.0 * float(ra.eps)
        nn_after, _, _ = model.top2(p1)
        failed = set(np.flatnonzero(nn_after != nn_before).tolist())
        assert failed <= ca <= cb
        a.repair()
        assert np.array_equal(a.nn, nn_after)
        n_cases += 1
        n_strict += len(cb - ca)
        n_boundary += int(np.sum(r == thr))
    assert n_cases == 504 * 125
    assert n_strict > 1000 and n_boundary > 1000


@pytest.mark.parametrize("d", [2, 3])
def test_budget_rule_multistep_lattice_walks_no_miss(d):
    """Random walks of 40 points on a fine dyadic lattice (exact arithmetic, ties
    everywhere), 30 steps each, with repairs and an occasional rebuild: refreshed keys
    carried over many steps never hide a failure."""
    g = np.random.default_rng(500 + d)
    for walk in range(12):
        p = (g.integers(0, 16, (d, 40)) / 16.0).astype(np.float64)
        sc = model.OracleScene(d=d, n=40, G=4, guard=0.0 if walk % 2 else model.GUARD_DEFAULT, rule="budget")
        sc.init_certificates(p.astype(np.float32))
        for t in range(30):
            mv = np.zeros_like(p)
            who = g.random(40) < 0.3
            ax = g.integers(0, d, 40)
            mv[ax, np.arange(40)] = np.where(who, g.choice([-1.0, 1.0], 40) / 64.0, 0.0)
            p = p + mv
            nn_before = sc.nn.copy()
            res = sc.step(p.astype(np.float32))
            nn_after, _, _ = model.top2(p.astype(np.float32))
            assert set(np.flatnonzero(nn_after != nn_before).tolist()) <= set(res.candidates.tolist())
            sc.rebuild() if t % 11 == 10 else sc.repair()
            assert np.array_equal(sc.nn, nn_after), (walk, t)


@pytest.mark.parametrize("family", ["uniform_brownian", "ring_rotation", "adversarial_crossing", "clustered_drift",
                                    "shear_band"])
def test_budget_rule_no_miss_on_the_workload_families(family):
    """Reduced cube trajectories (N = 3000, 25 steps): every step the per-point rule
    misses nothing, its failure set is the true change, and over the run it flags
    fewer points than the clock rule."""
    tr = synth.make_trajectory(family, 3000, 3, 25, 5e-4, 2000 + synth.FAMILIES.index(family))
    a = model.OracleScene(d=3, n=3000, G=9, rule="budget")
    b = model.OracleScene(d=3, n=3000, G=9)
    a.init_certificates(tr.frames[0])
    b.init_certificates(tr.frames[0])
    prev = a.nn.copy()
    na = nb = 0
    for t in range(1, 26):
        ra, rb = a.step(tr.frames[t]), b.step(tr.frames[t])
        a.repair()
        b.repair()
        now = model.top2(tr.frames[t])[0]
        assert np.array_equal(a.nn, now) and np.array_equal(b.nn, now)
        assert set(np.flatnonzero(a.fail)) == set(np.flatnonzero(now != prev))
        prev = now
        na += ra.candidates.size
        nb += rb.candidates.size
    assert na < nb


def test_gyration_closed_forms():
    """Radius of gyration of a frontier: two points 2a apart -> a; the 2^d corners of a
    cube of side 2a -> a sqrt(d); one point or none -> 0; invariant under translation."""
    for d in (2, 3):
        p = np.zeros((d, 2), np.float32)
        p[0, 1] = 0.5
        g, c = model.gyration(p, np.array([True, True]))
        assert g == 0.25 and c[0] == 0.25
        corners = np.array(list(itertools.product((0.25, 0.75), repeat=d)), np.float32).T
        g, c = model.gyration(corners, np.ones(2 ** d, bool))
        assert abs(g - 0.25 * math.sqrt(d)) < 1e-15 and np.allclose(c[:d], 0.5)
        g, _ = model.gyration(corners, np.array([3]))
        assert g == 0.0
        assert model.gyration(corners, np.zeros(2 ** d, bool))[0] == 0.0
        shifted = (corners + np.float32(0.125)).astype(np.float32)
        assert model.gyration(shifted, np.ones(2 ** d, bool))[0] == model.gyration(corners, np.ones(2 ** d, bool))[0]


def _block_scene(k_from, k_to, q_move=0.0):
    """Unit square, G = 4 (cells of 1/4): i = (0.625, 0.625) with j at distance 1/64 and
    m at 1/32 (all in cell (2, 2), whose block spans cells 1..3 on each axis: the
    distance from i to the block's outside is 0.375, the high sides being open); k
    moves on the line y = 0.625 from x = k_from to k_to; q, inside i's block at
    (0.875, 0.375) (cell (3, 1)), moves by q_move along y.  Values are dyadic."""
    p0 = np.array([[0.625, 0.625 + 1 / 64, 0.625, k_from, 0.875],
                   [0.625, 0.625, 0.625 + 1 / 32, 0.625, 0.375]])
    p1 = p0.copy()
    p1[0, 3] = k_to
    p1[1, 4] += q_move
    return p0.astype(np.float32), p1.astype(np.float32)


def test_budget_block_rule_constructions():
    """The block-local half of the budget: a quiet block with no reachable outsider
    keeps i's certificate although the clock rule flags it; a jump from outside the
    block that could reach within d2 makes i a candidate (and the failure is caught);
    a mover inside the block hands i over to the distance test."""
    cases = [  # (k_from, k_to, q_move, budget candidate, clock candidate, nn changes)
        (0.09375, 0.15625, 0.0, False, True, False),    # k moves 1/16 inside cell 0: quiet block
        (0.09375, 0.6171875, 0.0, True, True, True),    # k jumps next to i: 0.523 > B - d2
        (0.09375, 0.15625, 1 / 64, True, True, False),  # q moves inside the block, eps = 1/16
    ]
    for k_from, k_to, q_move, want_budget, want_clock, changes in cases:
        p0, p1 = _block_scene(k_from, k_to, q_move)
        for rule, want in (("budget", want_budget), ("clock", want_clock)):
            sc = model.OracleScene(d=2, n=5, G=4, guard=0.0, rule=rule)
            sc.init_certificates(p0)
            assert sc.nn[0] == 1 and float(sc.d2[0]) == 1 / 32
            res = sc.step(p1)
            assert (0 in set(res.candidates.tolist())) == want, (k_from, k_to, q_move, rule)
            sc.repair()
            assert bool(sc.fail[0]) == changes
            assert sc.audit().size == 0


def test_budget_rule_localized_motion_localizes_the_candidates():
    """Motion confined to one disc: under the budget rule every candidate lies within a
    block of a cell some moving point left or entered, the candidates are a strict
    subset of the clock rule's, and nothing is missed; motion of the same number of
    points spread uniformly makes many more candidates."""
    g = np.random.default_rng(77)
    n, G = 20000, 70
    p0 = g.random((2, n))
    centre = np.array([[0.3], [0.6]])
    inside = np.flatnonzero(np.hypot(*(p0 - centre)) < 0.08)
    spread = g.choice(n, inside.size, replace=False)
    counts = {}
    for name, movers in (("localized", inside), ("diffuse", spread)):
        p1 = p0.copy()
        step = g.standard_normal((2, movers.size))
        p1[:, movers] += 2e-4 * step / np.linalg.norm(step, axis=0)
        a = model.OracleScene(d=2, n=n, G=G, rule="budget")
        b = model.OracleScene(d=2, n=n, G=G)
        a.init_certificates(p0.astype(np.float32))
        b.init_certificates(p0.astype(np.float32))
        ca = set(a.step(p1.astype(np.float32)).candidates.tolist())
        cb = set(b.step(p1.astype(np.float32)).candidates.tolist())
        assert ca < cb
        stamped = np.flatnonzero(a.last_move == 1)
        sx, sy = stamped % G, stamped // G
        for i in ca:
            gx, gy = a.cell[i] % G, a.cell[i] // G
            assert np.any((np.abs(sx - gx) <= 1) & (np.abs(sy - gy) <= 1)), i
        a.repair()
        assert a.audit().size == 0
        counts[name] = len(ca)
    assert counts["diffuse"] > 3 * counts["localized"]
