"""Pins of the CPU oracle: checks against what the paper and the mathematics fix.

Each ``pin_*`` function takes a loaded oracle library and raises
AssertionError if the oracle disagrees with:
  - the worked example the paper prints (Table 1, figure "Stack vs. queue");
  - hand-derived special cases of Algorithm 1 (ties, diagonals, dx != dy);
  - brute force on tiny grids (path walks for levels and areas, a dense
    linear solve for the implicit height update of Algorithm 6);
  - closed forms: K = 0, very long time steps, the steady-state slope-area
    law S = (U/K) A^-m and the 1-D channel profile.
The same functions serve the mutation test, which plants mistakes in a copy
of the oracle and expects at least one pin to fail for each.
"""
from __future__ import annotations

import json
import os

import numpy as np

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

# Neighbour offsets (dy, dx) in the oracle's neighbour order.
OFFS = [(-1, -1), (-1, 0), (-1, 1), (0, -1), (0, 1), (1, -1), (1, 0), (1, 1)]


def _table1():
    with open(os.path.join(GOLDEN, "table1_example.json")) as f:
        return json.load(f)


# --------------------------------------------------------------------------
# Worked example (Table 1; figure "Stack vs. queue").

def pin_table1(lib):
    t = _table1()
    n = len(t["nodes"])
    rec = np.array([(r - 1) if r is not None else i for i, r in enumerate(t["rec"])], np.int32)
    g = oracle.graph_order(rec, lib=lib)
    assert g["dnum"].tolist() == t["dnum"], ("Dnum", g["dnum"].tolist())
    for node, dl in t["donors"].items():
        c = int(node) - 1
        got = [int(v) + 1 for v in g["donor"][c, : g["dnum"][c]]]
        assert got == dl, ("Donor", node, got, dl)
    assert (g["queue"] + 1).tolist() == t["queue"], ("Queue", (g["queue"] + 1).tolist())
    assert g["levels"].tolist() == t["levels"], ("Levels", g["levels"].tolist())
    assert g["count"].tolist() == t["accum"], ("Accum", g["count"].tolist())
    order = (g["stack_order"] + 1).tolist()
    expect = sorted(t["stack_visit_number"], key=lambda k: t["stack_visit_number"][k])
    assert order == [int(k) for k in expect], ("stack order", order)
    bfs = sorted(t["queue_visit_number"], key=lambda k: t["queue_visit_number"][k])
    assert (g["queue"] + 1).tolist() == [int(k) for k in bfs]
    # The levels of the queue are the depths of the nodes.
    for l in range(len(t["levels"]) - 1):
        for i in range(t["levels"][l], t["levels"][l + 1]):
            assert g["depth"][g["queue"][i]] == l
    assert n == 10


# --------------------------------------------------------------------------
# Receivers: hand-derived special cases of Algorithm 1.

def _rec_of(lib, h, dx=100.0, dy=100.0):
    return oracle.receivers(np.asarray(h, np.float64), dx, dy, lib=lib)


def pin_receivers_special_cases(lib):
    z = np.zeros((3, 3))
    # Centre above a flat perimeter: the four orthogonal slopes tie at 1/100
    # and beat the diagonals (1/141.4); the first in neighbour order (up) wins.
    h = z.copy(); h[1, 1] = 1.0
    assert _rec_of(lib, h)[1, 1] == 1
    # A lower diagonal corner beats the orthogonal neighbours: 2/141.4 > 1/100.
    h = z.copy(); h[1, 1] = 1.0; h[0, 0] = -1.0
    assert _rec_of(lib, h)[1, 1] == 0
    # ... but not when it is only slightly lower: 1.2/141.4 < 1/100.
    h = z.copy(); h[1, 1] = 1.0; h[2, 2] = -0.2
    assert _rec_of(lib, h)[1, 1] == 1
    # Flat and pit: no strictly lower neighbour, so no receiver.
    assert _rec_of(lib, z)[1, 1] == 4
    h = z.copy(); h[1, 1] = -1.0
    assert _rec_of(lib, h)[1, 1] == 4
    # dx != dy: with dx = 50 the left neighbour (slope 1/50) beats up (1/100).
    h = z.copy(); h[1, 1] = 1.0
    assert _rec_of(lib, h, dx=50.0, dy=100.0)[1, 1] == 3
    assert _rec_of(lib, h, dx=100.0, dy=50.0)[1, 1] == 1
    # Perimeter cells never have a receiver.
    h = np.arange(20, dtype=np.float64).reshape(4, 5)
    rec = _rec_of(lib, h)
    for y in range(4):
        for x in range(5):
            if y in (0, 3) or x in (0, 4):
                assert rec[y, x] == y * 5 + x
    # A plane rising in x drains every interior cell to its left neighbour;
    # a plane rising in x and y drains to the upper-left diagonal.
    yy, xx = np.mgrid[0:6, 0:7].astype(np.float64)
    rec = _rec_of(lib, xx)
    for y in range(1, 5):
        for x in range(1, 6):
            assert rec[y, x] == y * 7 + x - 1
    rec = _rec_of(lib, xx + yy)
    for y in range(1, 5):
        for x in range(1, 6):
            assert rec[y, x] == (y - 1) * 7 + x - 1


def _receivers_brute(h, dx, dy):
    """Every slope of every interior cell at once; the first maximum wins."""
    ny, nx = h.shape
    dd = np.sqrt(dx * dx + dy * dy)
    dist = [dd, dy, dd, dx, dx, dd, dy, dd]
    rec = np.arange(ny * nx, dtype=np.int64).reshape(ny, nx)
    if ny < 3 or nx < 3:
        return rec
    hc = h[1:-1, 1:-1]
    s = np.stack([(hc - h[1 + oy: ny - 1 + oy, 1 + ox: nx - 1 + ox]) / dist[k]
                  for k, (oy, ox) in enumerate(OFFS)])
    best = np.argmax(s, axis=0)
    smax = np.take_along_axis(s, best[None], 0)[0]
    iy, ix = np.mgrid[1:ny - 1, 1:nx - 1]
    oy = np.array([o[0] for o in OFFS])[best]
    ox = np.array([o[1] for o in OFFS])[best]
    target = (iy + oy) * nx + (ix + ox)
    rec[1:-1, 1:-1] = np.where(smax > 0.0, target, iy * nx + ix)
    return rec


def pin_receivers_brute_force(lib):
    rng = np.random.default_rng(11)
    for trial in range(40):
        ny = int(rng.integers(3, 10))
        nx = int(rng.integers(3, 10))
        h = W.quantised_heights(ny, nx, 4, seed=1000 + trial)
        dx = float(rng.choice([1.0, 30.0, 100.0]))
        dy = dx if trial % 2 == 0 else float(rng.choice([20.0, 70.0]))
        got = _rec_of(lib, h, dx, dy)
        exp = _receivers_brute(h, dx, dy)
        assert np.array_equal(got, exp), (trial, ny, nx, dx, dy)


# --------------------------------------------------------------------------
# Levels and areas: path-walk brute force and invariants.

def _walk(rec):
    """Each cell walks to its root: its depth is the number of hops, and it
    adds one to the count of every cell on the way (itself included)."""
    r = rec.ravel()
    n = r.size
    depth = np.zeros(n, np.int64)
    count = np.zeros(n, np.int64)
    for c in range(n):
        v, d = c, 0
        count[v] += 1
        while r[v] != v:
            v = r[v]
            d += 1
            count[v] += 1
            assert d <= n
        depth[c] = d
    return depth, count


def pin_levels_and_areas_brute_force(lib):
    for seed, (ny, nx, q) in enumerate([(7, 9, 3), (12, 10, 5), (16, 16, 0), (5, 23, 2)]):
        h = (W.quantised_heights(ny, nx, q, seed) if q else W.initial_heights(ny, nx, seed))
        p = oracle.Params(ny, nx)
        r = oracle.routing(h, p, lib=lib)
        depth, count = _walk(r["rec"])
        assert np.array_equal(r["depth"].ravel(), depth), (ny, nx)
        assert np.array_equal(r["count"].ravel(), count), (ny, nx)
        hist = np.bincount(depth, minlength=r["nlevels"])
        assert r["nlevels"] == depth.max() + 1
        assert np.array_equal(r["offsets"], np.concatenate([[0], np.cumsum(hist)]))


def pin_forest_invariants(lib):
    h = W.initial_heights(40, 33, 5)
    p = oracle.Params(40, 33)
    r = oracle.routing(h, p, lib=lib)
    rec = r["rec"].ravel()
    cnt = r["count"].ravel().astype(np.int64)
    dep = r["depth"].ravel()
    n = rec.size
    roots = rec == np.arange(n)
    assert cnt[roots].sum() == n
    assert np.all(dep[roots] == 0)
    nr = ~roots
    assert np.all(dep[nr] == dep[rec[nr]] + 1)
    inflow = np.zeros(n, np.int64)
    np.add.at(inflow, rec[nr], cnt[nr])
    assert np.array_equal(cnt, 1 + inflow)
    # In depth-first order every subtree is one contiguous block of
    # count[c] cells that starts at c.
    donor, dnum = oracle.donors(r["rec"], lib=lib)
    order, depth, emitted = oracle.stack_order(r["rec"], donor, dnum, lib=lib)
    assert emitted == n
    pos = np.empty(n, np.int64)
    pos[order] = np.arange(n)
    def has_ancestor(v, c):
        while v != c and rec[v] != v:
            v = rec[v]
        return v == c

    for c in range(n):
        block = order[pos[c]: pos[c] + cnt[c]]
        assert all(has_ancestor(int(v), c) for v in block), c
    # The breadth-first queue of Algorithm 3 has exactly these levels.
    queue, levels = oracle.bfs_queue(r["rec"], donor, dnum, lib=lib)
    assert np.array_equal(levels, r["offsets"])
    for l in range(len(levels) - 1):
        assert np.all(dep[queue[levels[l]: levels[l + 1]]] == l)


# --------------------------------------------------------------------------
# Heights: brute force and closed forms.

def _dist(c, r, nx, dx, dy):
    cy, cx, ry, rx = c // nx, c % nx, r // nx, r % nx
    if cy != ry and cx != rx:
        return np.sqrt(dx * dx + dy * dy)
    return dy if cy != ry else dx


def pin_one_step_dense_solve(lib):
    """Backward Euler for every cell at once: (I + diag(F)(I - P)) h' = h + U dt."""
    for seed, (ny, nx, m, Kfield) in enumerate([(6, 7, 0.5, False), (8, 5, 0.45, True),
                                                (9, 9, 0.6, False)]):
        dx, dy, dt, U, K = 30.0, 45.0, 1e4, 2e-3, 4e-5
        h = W.initial_heights(ny, nx, 50 + seed) * 5.0
        Kf = (K * np.exp(0.5 * np.random.default_rng(seed).standard_normal((ny, nx)))
              if Kfield else None)
        Uf = np.random.default_rng(seed + 7).uniform(1e-4, 2e-3, (ny, nx))
        p = oracle.Params(ny, nx, dx, dy, dt, m, 1.0, U, K)
        rec = _receivers_brute(h, dx, dy).ravel()
        _, count = _walk(rec.reshape(ny, nx))
        n = ny * nx
        A = np.eye(n)
        rhs = h.ravel().copy()
        for c in range(n):
            y, x = divmod(c, nx)
            interior = 0 < y < ny - 1 and 0 < x < nx - 1
            if interior:
                rhs[c] += Uf.ravel()[c] * dt
            if rec[c] != c:
                kc = Kf.ravel()[c] if Kfield else K
                F = kc * dt * (count[c] * dx * dy) ** m / _dist(c, rec[c], nx, dx, dy)
                A[c, c] += F
                A[c, rec[c]] -= F
        exp = np.linalg.solve(A, rhs).reshape(ny, nx)
        got = oracle.run(h, p, 1, K=Kf, U=Uf, lib=lib)["h"]
        assert np.allclose(got, exp, rtol=1e-12, atol=1e-12), (seed, np.abs(got - exp).max())


def pin_no_erosion_is_pure_uplift(lib):
    h = W.initial_heights(20, 17, 9)
    p = oracle.Params(20, 17, 100.0, 100.0, 1000.0, 0.5, 1.0, 5e-4, 0.0)
    got = oracle.run(h, p, 3, lib=lib)["h"]
    exp = h.copy()
    for _ in range(3):
        exp[1:-1, 1:-1] = exp[1:-1, 1:-1] + 5e-4 * 1000.0
    assert np.array_equal(got, exp)


def pin_long_step_follows_receiver(lib):
    """As dt grows, F grows and every eroding cell moves onto its receiver's
    new height; roots keep only the uplift."""
    h = W.initial_heights(12, 14, 21)
    p = oracle.Params(12, 14, 100.0, 100.0, 1e9, 0.5, 1.0, 0.0, 1.0)
    r = oracle.routing(h, p, lib=lib)
    got = oracle.run(h, p, 1, lib=lib)["h"].ravel()
    rec = r["rec"].ravel()
    for c in range(rec.size):
        root = c
        while rec[root] != root:
            root = rec[root]
        assert abs(got[c] - got[root]) < 1e-6, c


def _run_to_steady(lib, h, p, rec=None, block=200, max_blocks=200):
    for _ in range(max_blocks):
        if rec is None:
            nxt = oracle.run(h, p, block, lib=lib)["h"]
        else:
            nxt = oracle.run_fixed_routing(h, rec, p, block, lib=lib)["h"]
        change = np.abs(nxt - h).max() / max(np.abs(nxt).max(), 1e-300)
        h = nxt
        if change < 1e-14:
            return h
    raise AssertionError("no steady state")


def pin_steady_state_slope_area(lib):
    """At the fixed point of uplift and implicit erosion every cell satisfies
    U dt = F (h_c - h_r), i.e. S = (h_c - h_r)/d = (U/K) A^-m, whatever dt."""
    ny = nx = 24
    yy, xx = np.mgrid[0:ny, 0:nx]
    cone = np.minimum.reduce([yy, xx, ny - 1 - yy, nx - 1 - xx]).astype(np.float64)
    h = cone + 0.3 * np.random.default_rng(4).random((ny, nx))
    h[0, :] = h[-1, :] = h[:, 0] = h[:, -1] = 0.0
    U, K, m, dx = 1e-3, 2e-5, 0.45, 30.0
    p = oracle.Params(ny, nx, dx, dx, 5e4, m, 1.0, U, K)
    h = _run_to_steady(lib, h, p)
    r = oracle.routing(h, p, lib=lib)
    rec, cnt = r["rec"].ravel(), r["count"].ravel()
    hf = h.ravel()
    checked = 0
    for c in range(hf.size):
        y, x = divmod(c, nx)
        if not (0 < y < ny - 1 and 0 < x < nx - 1):
            continue
        assert rec[c] != c, "an interior sink survived"
        S = (hf[c] - hf[rec[c]]) / _dist(c, rec[c], nx, dx, dx)
        law = (U / K) * (cnt[c] * dx * dx) ** (-m)
        assert abs(S - law) <= 1e-9 * law, (c, S, law)
        checked += 1
    assert checked == (ny - 2) * (nx - 2)


def pin_channel_profile(lib):
    """A 1-D channel (fixed routing: every interior cell of the middle row
    drains left) reaches h_i = sum_{j<=i} dx (U/K) A_j^-m, A_j = (nx-1-j) dx dy."""
    ny, nx = 3, 40
    U, K, m, dx, dy = 5e-4, 1e-5, 0.5, 100.0, 100.0
    rec = np.arange(ny * nx, dtype=np.int32).reshape(ny, nx)
    for x in range(1, nx - 1):
        rec[1, x] = nx + x - 1
    p = oracle.Params(ny, nx, dx, dy, 1e5, m, 1.0, U, K)
    h = _run_to_steady(lib, np.zeros((ny, nx)), p, rec=rec)
    expect = np.cumsum([dx * (U / K) * ((nx - 1 - j) * dx * dy) ** (-m) for j in range(1, nx - 1)])
    assert np.allclose(h[1, 1:-1], expect, rtol=1e-10, atol=0), np.abs(h[1, 1:-1] - expect).max()
    assert np.all(h[0] == 0) and np.all(h[2] == 0)


def pin_newton_matches_closed_form(lib):
    """Algorithm 6's Newton loop with n = 1 converges to the closed form."""
    h = W.initial_heights(30, 30, 2) * 3
    p1 = oracle.Params(30, 30, m=0.5, n=1.0)
    pn = oracle.Params(30, 30, m=0.5, n=1.0 + 1e-15)
    a = oracle.run(h, p1, 5, lib=lib)["h"]
    b = oracle.run(h, pn, 5, lib=lib)["h"]
    assert np.allclose(a, b, rtol=1e-12, atol=1e-12)


def pin_newton_channel_profile(lib):
    """Slope exponent n != 1 (Algorithm 6's Newton loop): at steady state
    K A^m S^n = U, so a 1-D channel reaches h_i = sum_{j<=i} dx (U/(K A_j^m))^(1/n)."""
    ny, nx = 3, 30
    U, K, m, dx, dy = 5e-4, 1e-5, 0.5, 100.0, 100.0
    rec = np.arange(ny * nx, dtype=np.int32).reshape(ny, nx)
    for x in range(1, nx - 1):
        rec[1, x] = nx + x - 1
    for nexp in (2.0, 1.5, 0.8):
        p = oracle.Params(ny, nx, dx, dy, 1e4, m, nexp, U, K, eps=1e-10)
        h = _run_to_steady(lib, np.zeros((ny, nx)), p, rec=rec)
        expect = np.cumsum([dx * (U / (K * ((nx - 1 - j) * dx * dy) ** m)) ** (1.0 / nexp)
                            for j in range(1, nx - 1)])
        assert np.allclose(h[1, 1:-1], expect, rtol=1e-9, atol=0), (nexp, np.abs(h[1, 1:-1] - expect).max())


def pin_newton_step_solves_the_implicit_equation(lib):
    """One step with n = 2: every non-root cell satisfies the backward-Euler
    equation h'_c = h_c + U dt - K dt A^m ((h'_c - h'_r)/d)^n up to the
    Newton tolerance, with h'_r the receiver's new height."""
    ny, nx = 20, 26
    h = W.initial_heights(ny, nx, 6) * 50.0
    dx, dy, nexp, eps = 40.0, 70.0, 2.0, 1e-12
    p = oracle.Params(ny, nx, dx, dy, 2000.0, 0.45, nexp, 1e-3, 3e-5, eps=eps)
    rec = oracle.receivers(h, dx, dy, lib=lib)
    out = oracle.run_fixed_routing(h, rec, p, 1, lib=lib)
    hn, cnt = out["h"].ravel(), out["count"].ravel()
    recf, h0 = rec.ravel(), h.ravel()
    checked = 0
    for c in range(h0.size):
        r = recf[c]
        if r == c:
            continue
        d = _dist(c, r, nx, dx, dy)
        f = p.K * p.dt * (cnt[c] * dx * dy) ** p.m / d ** nexp
        gap = hn[c] - hn[r]
        assert gap > 0, (c, gap)
        res = hn[c] - (h0[c] + p.U * p.dt) + f * gap ** nexp
        assert abs(res) <= 10 * eps * (1 + f * nexp * gap ** (nexp - 1)) + 1e-13 * abs(hn[c]), (c, res)
        checked += 1
    assert checked > 0


def _chain_routing(ny, nx):
    """Fixed routing of a 1-D channel: every interior cell of the middle row
    drains to its left neighbour; the left perimeter cell is the outlet."""
    rec = np.arange(ny * nx, dtype=np.int32).reshape(ny, nx)
    for x in range(1, nx - 1):
        rec[1, x] = nx + x - 1
    return rec


def _newton_cells(h_in, out, rec, p, U):
    """(c, h0, hr', F, h') for every non-root cell of a fixed-routing step."""
    nx = p.nx
    hn, cnt = out["h"].ravel(), out["count"].ravel()
    recf, hin, uf = rec.ravel(), h_in.ravel(), np.ravel(U)
    for c in range(hin.size):
        r = recf[c]
        if r == c:
            continue
        d = _dist(c, r, nx, p.dx, p.dy)
        f = p.K * p.dt * (cnt[c] * p.dx * p.dy) ** p.m / d ** p.n
        yield c, hin[c] + uf[c] * p.dt, hn[r], f, hn[c]


def pin_newton_overshoot_stays_above_receiver(lib):
    """n = 0.5 with a large F: the first Newton iterate from h0 falls below the
    receiver for some cells.  The backward-Euler equation
    h' - h0 + F (h' - h'_r)^n = 0 still has exactly one root in (h'_r, h0];
    every cell's new height must be that root (found here by SciPy's brentq),
    strictly above its receiver."""
    from scipy.optimize import brentq
    ny, nx = 3, 24
    rec = _chain_routing(ny, nx)
    h = np.zeros((ny, nx))
    h[1, 1:-1] = np.linspace(0.4, 9.0, nx - 2)
    p = oracle.Params(ny, nx, 100.0, 100.0, 5e4, 0.5, 0.5, 1e-4, 4e-5, eps=1e-13, max_newton=200)
    U = np.full((ny, nx), p.U)
    out = oracle.run_fixed_routing(h, rec, p, 1, U=U, lib=lib)
    overshoots = 0
    for c, h0, hr, f, got in _newton_cells(h, out, rec, p, U):
        g = h0 - hr
        first = h0 - (f * g ** p.n) / (1.0 + f * p.n * g ** (p.n - 1.0))
        overshoots += first <= hr
        assert got > hr, (c, got, hr)
        root = brentq(lambda x: x - h0 + f * (x - hr) ** p.n, hr, h0, xtol=1e-15, rtol=1e-15)
        assert abs(got - root) <= 1e-10 * max(abs(root), 1.0), (c, got, root)
    assert overshoots >= 3, overshoots
    # An iterate landing exactly on the receiver: h0 = 1 above an outlet at 0,
    # F = K dt A^m / d^n = 0.5 * 4 * 1 / 1 = 2 and n = 0.5 give the first step
    # 1 - 2 / (1 + 0.5 * 2) = 0 exactly; the root is (sqrt(2) - 1)^2.
    rec = _chain_routing(3, 3)
    h = np.zeros((3, 3))
    h[1, 1] = 1.0
    p = oracle.Params(3, 3, 1.0, 1.0, 4.0, 0.5, 0.5, 0.0, 0.5, eps=1e-15, max_newton=200)
    got = oracle.run_fixed_routing(h, rec, p, 1, lib=lib)["h"][1, 1]
    assert abs(got - (np.sqrt(2.0) - 1.0) ** 2) <= 1e-14, got


def pin_newton_iteration_cap(lib):
    """n = 2 with one permitted iteration: the residual is convex, so Newton
    from h0 approaches the root from above; after one iteration each cell
    with a noticeable slope lies strictly between the exact root (brentq)
    and h0."""
    from scipy.optimize import brentq
    ny, nx = 3, 16
    rec = _chain_routing(ny, nx)
    h = np.zeros((ny, nx))
    h[1, 1:-1] = np.linspace(2.0, 30.0, nx - 2)
    p = oracle.Params(ny, nx, 100.0, 100.0, 1e4, 0.5, 2.0, 1e-4, 2e-4, eps=1e-14, max_newton=1)
    U = np.full((ny, nx), p.U)
    out = oracle.run_fixed_routing(h, rec, p, 1, U=U, lib=lib)
    checked = 0
    for c, h0, hr, f, got in _newton_cells(h, out, rec, p, U):
        root = brentq(lambda x: x - h0 + f * (x - hr) ** 2, hr, h0, xtol=1e-15, rtol=1e-15)
        assert root < got < h0, (c, root, got, h0)
        assert got - root > 1e-6 * (h0 - root), (c, got, root)
        checked += 1
    assert checked == nx - 2


def pin_newton_cell_not_above_receiver_keeps_height(lib):
    """A U field that lifts a receiver above its donor: the donor has no
    positive slope, so no erosion applies and it keeps its uplifted height
    exactly; the cells that stay above their receivers erode."""
    ny, nx = 3, 6
    rec = _chain_routing(ny, nx)
    h = np.zeros((ny, nx))
    h[1, 1:-1] = [1.0, 2.0, 3.0, 4.0]
    U = np.zeros((ny, nx))
    U[1, 2] = 0.01  # the receiver of cell (1, 3) rises by 10 m
    p = oracle.Params(ny, nx, 100.0, 100.0, 1e3, 0.5, 1.5, 0.0, 1e-6, eps=1e-12, max_newton=50)
    out = oracle.run_fixed_routing(h, rec, p, 1, U=U, lib=lib)
    hn = out["h"]
    assert hn[1, 3] == 3.0, hn[1, 3]
    assert hn[1, 2] > hn[1, 3]
    assert 0.0 < hn[1, 1] < 1.0 and 3.0 < hn[1, 4] < 4.0, hn[1]


def _mfd_receivers(h, dx, dy, pexp):
    """Receivers and shares of every interior cell by the definition:
    strictly lower neighbours, share proportional to slope**pexp."""
    ny, nx = h.shape
    out = {}
    for y in range(1, ny - 1):
        for x in range(1, nx - 1):
            c = y * nx + x
            recs = []
            for k, (oy, ox) in enumerate(_NB):
                r = (y + oy) * nx + (x + ox)
                if h.flat[c] - h.flat[r] > 0:
                    d = _dist(c, r, nx, dx, dy)
                    recs.append((r, ((h.flat[c] - h.flat[r]) / d) ** pexp, d))
            tot = sum(w for _, w, _ in recs)
            out[c] = [(r, w / tot, d) for r, w, d in recs]
    return out


_NB = [(-1, -1), (-1, 0), (-1, 1), (0, -1), (0, 1), (1, -1), (1, 0), (1, 1)]


def pin_mfd_area_conservation_and_dense_solve(lib):
    """Multiple flow directions: every cell's area ends at a cell without
    receivers (shares sum to one), and the areas solve the linear system
    A_c = dx dy + sum_d s_{d->c} A_d whatever the processing order."""
    for seed, quant in ((1, None), (2, 3)):
        ny, nx = 7, 9
        h = (W.initial_heights(ny, nx, seed) if quant is None
             else W.quantised_heights(ny, nx, quant, seed))
        dx, dy, pexp = 30.0, 45.0, (1.0 if quant else 1.3)
        p = oracle.Params(ny, nx, dx, dy, 1000.0, 0.5, 1.0, 1e-3, 0.0)
        r = oracle.mfd_run(h, p, 1, pexp=pexp, lib=lib)
        A = r["area"].ravel()
        recs = _mfd_receivers(h, dx, dy, pexp)
        roots = [c for c in range(ny * nx) if not recs.get(c)]
        total = ny * nx * dx * dy
        assert abs(sum(A[c] for c in roots) - total) <= 1e-12 * total
        M = np.eye(ny * nx)
        for d, lst in recs.items():
            for c, s, _ in lst:
                M[c, d] -= s
        ref = np.linalg.solve(M, np.full(ny * nx, dx * dy))
        assert np.allclose(A, ref, rtol=1e-12, atol=0)


def pin_mfd_levels_are_longest_paths(lib):
    """The level of a cell is the length of the longest descending path from
    it to a cell without receivers (brute-force relaxation)."""
    ny, nx = 8, 8
    h = W.quantised_heights(ny, nx, 5, 9)
    p = oracle.Params(ny, nx)
    lev = oracle.mfd_run(h, p, 1, lib=lib)["level"].ravel()
    recs = _mfd_receivers(h, 100.0, 100.0, 1.0)
    ref = np.zeros(ny * nx, int)
    for _ in range(ny * nx):
        for c, lst in recs.items():
            for r, _, _ in lst:
                ref[c] = max(ref[c], ref[r] + 1)
    assert np.array_equal(lev, ref)


def pin_mfd_step_solves_the_implicit_system(lib):
    """One step with K > 0: the new heights solve (1 + sum F) h_c - sum F_k
    h_k = h_c + U dt (dense solve), F_k = K dt (s_k A_c)^m / d_k; cells
    without receivers are only uplifted and the perimeter stays put."""
    ny, nx = 7, 8
    h = W.initial_heights(ny, nx, 4) * 20.0
    dx, dy, pexp, m = 50.0, 40.0, 1.1, 0.45
    p = oracle.Params(ny, nx, dx, dy, 3000.0, m, 1.0, 2e-3, 3e-5)
    r = oracle.mfd_run(h, p, 1, pexp=pexp, lib=lib)
    A = r["area"].ravel()
    recs = _mfd_receivers(h, dx, dy, pexp)
    n = ny * nx
    M = np.eye(n)
    rhs = h.ravel().copy()
    for c, lst in recs.items():
        rhs[c] += p.U * p.dt
        for rr, s, d in lst:
            f = p.K * p.dt * (s * A[c]) ** m / d
            M[c, c] += f
            M[c, rr] -= f
    ref = np.linalg.solve(M, rhs)
    assert np.allclose(r["h"].ravel(), ref, rtol=1e-12, atol=1e-12)


def pin_mfd_without_erosion_is_pure_uplift(lib):
    h = W.initial_heights(9, 11, 5)
    p = oracle.Params(9, 11, K=0.0, U=2e-3)
    got = oracle.mfd_run(h, p, 3, lib=lib)["h"]
    ref = h.copy()
    ref[1:-1, 1:-1] += 3 * (2e-3 * 1000.0)
    assert np.allclose(got, ref, rtol=0, atol=1e-12)


def pin_projection_solves_the_steady_equation(lib):
    """One steady-state projection with fields: every cell with a receiver
    satisfies F (h_c - h_r)^n = U_c dt with the routing of the heights it
    started from and F of Algorithm 6, each receiver's new height on the
    right; cells without a receiver are only uplifted."""
    ny, nx = 23, 31
    rng = np.random.default_rng(11)
    h0 = W.initial_heights(ny, nx, 5) * 7.0
    K = 1e-5 * np.exp(0.5 * rng.standard_normal((ny, nx)))
    U = rng.uniform(1e-4, 2e-3, (ny, nx))
    for nexp in (1.0, 1.5):
        p = oracle.Params(ny, nx, 100.0, 70.0, 1e4, 0.45, nexp, 0.0, 1e-5)
        r0 = oracle.routing(h0, p, lib=lib)
        out = oracle.project(h0, p, 1, K=K, U=U, lib=lib)
        assert np.array_equal(out["rec"], r0["rec"])
        rec, cnt = r0["rec"].ravel(), r0["count"].ravel()
        a, b = out["h"].ravel(), h0.ravel()
        checked = 0
        for c in range(a.size):
            y, x = divmod(c, nx)
            if not (0 < y < ny - 1 and 0 < x < nx - 1):
                assert a[c] == b[c]
                continue
            udt = U.ravel()[c] * p.dt
            if rec[c] == c:
                assert a[c] == b[c] + udt
                continue
            d = _dist(c, rec[c], nx, p.dx, p.dy)
            F = K.ravel()[c] * p.dt * (cnt[c] * p.dx * p.dy) ** p.m / d ** nexp
            lhs = F * (a[c] - a[rec[c]]) ** nexp
            assert abs(lhs - udt) <= 1e-11 * udt, (nexp, c, lhs, udt)
            checked += 1
        assert checked > 0.8 * (ny - 2) * (nx - 2)


def pin_projection_fixed_point_is_a_steady_state(lib):
    """Repeated projections from a noisy cone stop changing; the result obeys
    the slope-area law S = (U/K) A^-m on every interior cell and one step of
    the method (uplift and implicit erosion) leaves it unchanged."""
    ny = nx = 24
    yy, xx = np.mgrid[0:ny, 0:nx]
    cone = np.minimum.reduce([yy, xx, ny - 1 - yy, nx - 1 - xx]).astype(np.float64)
    h = cone + 0.3 * np.random.default_rng(4).random((ny, nx))
    h[0, :] = h[-1, :] = h[:, 0] = h[:, -1] = 0.0
    U, K, m, dx = 1e-3, 2e-5, 0.45, 30.0
    p = oracle.Params(ny, nx, dx, dx, 5e3, m, 1.0, U, K)
    for _ in range(400):
        nxt = oracle.project(h, p, 1, lib=lib)["h"]
        change = np.abs(nxt - h).max() / np.abs(nxt).max()
        h = nxt
        if change == 0.0:
            break
    assert change == 0.0, change
    r = oracle.routing(h, p, lib=lib)
    rec, cnt, hf = r["rec"].ravel(), r["count"].ravel(), h.ravel()
    for c in range(hf.size):
        y, x = divmod(c, nx)
        if not (0 < y < ny - 1 and 0 < x < nx - 1):
            continue
        assert rec[c] != c, "an interior sink survived"
        S = (hf[c] - hf[rec[c]]) / _dist(c, rec[c], nx, dx, dx)
        law = (U / K) * (cnt[c] * dx * dx) ** (-m)
        assert abs(S - law) <= 1e-9 * law, (c, S, law)
    stepped = oracle.run(h, p, 1, lib=lib)["h"]
    assert np.abs(stepped - h).max() <= 1e-12 * np.abs(h).max()


ALL_PINS = [pin_table1, pin_receivers_special_cases, pin_receivers_brute_force,
            pin_levels_and_areas_brute_force, pin_forest_invariants, pin_one_step_dense_solve,
            pin_no_erosion_is_pure_uplift, pin_long_step_follows_receiver,
            pin_steady_state_slope_area, pin_channel_profile, pin_newton_matches_closed_form,
            pin_newton_channel_profile, pin_newton_step_solves_the_implicit_equation,
            pin_newton_overshoot_stays_above_receiver, pin_newton_iteration_cap,
            pin_newton_cell_not_above_receiver_keeps_height,
            pin_mfd_area_conservation_and_dense_solve, pin_mfd_levels_are_longest_paths,
            pin_mfd_step_solves_the_implicit_system, pin_mfd_without_erosion_is_pure_uplift,
            pin_projection_solves_the_steady_equation,
            pin_projection_fixed_point_is_a_steady_state]
