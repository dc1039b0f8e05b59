"""Pin of the binary64 decisions of the naive replica (oracle.naive.classify).

Sec. 4 evaluates Eq. 2.2 directly in binary64, and Sec. 2's existence test and the
containment rule are then decided on binary64 values.  Away from ties, i.e. where every
exact predicate value is far larger than the rounding error of its binary64 evaluation, a
correct binary64 classification must give exactly the exact oracle's answer (count, roots in
along-arc order, flags).  This pins the replica against ``geometry.classify``, whose own pins
are closed forms, brute-force sampling and exhaustive small-integer arcs.

The sample covers all four branches of the hit rule (monotone up and down, apex and nadir
inside), with hits and misses in each, and the mutants below (swapped heights, a flipped
slope, a flipped existence test, swapped root labels, a dropped branch) must each change at
least one well-conditioned answer.
"""

import inspect

import numpy as np
import pytest

from oracle import geometry as G
from oracle import naive
from paper_2510_09892_amd import inputs

MARGIN = 2.0 ** -24  # relative size of an exact predicate value that counts as "far from 0"


def _rel(v, scale):
    return abs(v) > MARGIN * scale if scale else False


def _well_conditioned(x1, x2, z0):
    """True when every predicate the hit rule reads is far from a tie (exact integers)."""
    t = G.exact_terms(x1, x2, z0)
    K = t["K"]
    Nx, Ny, Nz, S2, S3 = t["Nx"], t["Ny"], t["Nz"], t["S2"], t["S3"]
    if S2 == 0 or not _rel(S2, S3):
        return False
    # s^2 = S2 2^(2K) - S3 Z0^2 against its two terms
    if not _rel(t["s2"], (S2 << (2 * K)) + S3 * t["Z0"] ** 2):
        return False
    for X, Y, Z in ((t["X1"], t["Y1"], t["Z1"]), (t["X2"], t["Y2"], t["Z2"])):
        d = Nx * Y - Ny * X
        if not _rel(d, abs(Nx * Y) + abs(Ny * X)):
            return False
        # z0 against the endpoint's raw and normalised height: both must be far apart
        h = t["Z0"] ** 2 * (X * X + Y * Y + Z * Z) - (Z * Z << (2 * K))
        if not _rel(h, t["Z0"] ** 2 * (X * X + Y * Y + Z * Z) + (Z * Z << (2 * K))):
            return False
        if t["Z0"] == 0 or Z == 0:
            return False
    return True


def _branch(x1, x2, z0):
    t = G.exact_terms(x1, x2, z0)
    d1 = np.sign(t["Nx"] * t["Y1"] - t["Ny"] * t["X1"])
    d2 = np.sign(t["Nx"] * t["Y2"] - t["Ny"] * t["X2"])
    if d1 >= 0 and d2 >= 0:
        return "up"
    if d1 <= 0 and d2 <= 0:
        return "down"
    return "apex" if d1 > 0 else "nadir"


def _sample():
    """Uniform workload pairs, longer arcs (apex/nadir cases) and latitudes placed inside,
    around and away from each arc's height range."""
    out = []
    P = inputs.uniform_arcs(1500, seed_tag=41)
    out += list(zip(P.p1, P.p2, P.z0))
    g = inputs.rng(42)
    for d_hi in (0.2, 2.5):
        n = 1500
        p1 = inputs.random_unit(g, n)
        p2 = inputs.arc_from(p1, g.uniform(1e-3, d_hi, n), g.uniform(0, 2 * np.pi, n))
        lo, hi = inputs.z_range(p1, p2)
        w = hi - lo
        z_around = lo - w + 3 * w * g.random(n)  # a third below, a third inside, a third above
        z_any = g.uniform(-1, 1, n)
        out += list(zip(p1, p2, z_around)) + list(zip(p1, p2, z_any))
    return [(tuple(map(float, a)), tuple(map(float, b)), float(z)) for a, b, z in out]


@pytest.fixture(scope="module")
def pinned_pairs():
    pairs = _sample()
    good = [p for p in pairs if _well_conditioned(*p)]
    return pairs, good, [G.classify(*p) for p in good]


def _mismatches(classify, good, exact):
    bad = 0
    for p, c in zip(good, exact):
        cnt, roots, flags = classify(*p)
        if (cnt, roots, flags) != (c.count, c.roots, c.flags):
            bad += 1
    return bad


def test_naive_decisions_equal_exact_away_from_ties(pinned_pairs):
    pairs, good, exact = pinned_pairs
    # nearly every pair of these workloads is far from a tie
    assert len(good) >= 0.97 * len(pairs), (len(good), len(pairs))
    assert _mismatches(naive.classify, good, exact) == 0
    # the pin exercises every branch of the rule with hits and with misses, and 2-hit pairs
    seen = {}
    for p, c in zip(good, exact):
        key = (_branch(*p), c.count)
        seen[key] = seen.get(key, 0) + 1
    for br in ("up", "down", "apex", "nadir"):
        assert seen.get((br, 0), 0) >= 20, (br, seen)
        assert seen.get((br, 1), 0) >= 20, (br, seen)
    assert seen.get(("apex", 2), 0) >= 20 and seen.get(("nadir", 2), 0) >= 20, seen


MUTANTS = {
    "heights swapped": [("c1 = _sgn(z0 - x1[2])", "c1 = _sgn(z0 - x2[2])"),
                        ("c2 = _sgn(z0 - x2[2])", "c2 = _sgn(z0 - x1[2])")],
    "first slope flipped": [("d1 = _sgn(nx * x1[1] - ny * x1[0])",
                             "d1 = _sgn(ny * x1[0] - nx * x1[1])")],
    "second slope flipped": [("d2 = _sgn(nx * x2[1] - ny * x2[0])",
                              "d2 = _sgn(ny * x2[0] - nx * x2[1])")],
    "existence flipped": [("if s2 < 0.0:", "if s2 > 0.0:")],
    "monotone root label": [("roots = [PLUS] if (c1 >= 0 and c2 <= 0) else []",
                             "roots = [MINUS] if (c1 >= 0 and c2 <= 0) else []")],
    "apex order": [("roots = ([PLUS] if c1 >= 0 else []) + ([MINUS] if c2 >= 0 else [])",
                    "roots = ([MINUS] if c2 >= 0 else []) + ([PLUS] if c1 >= 0 else [])")],
    "nadir test": [("roots = ([MINUS] if c1 <= 0 else []) + ([PLUS] if c2 <= 0 else [])",
                    "roots = ([MINUS] if c1 >= 0 else []) + ([PLUS] if c2 <= 0 else [])")],
    "normal component": [("ny = x1[2] * x2[0] - x1[0] * x2[2]",
                          "ny = x1[0] * x2[2] - x1[2] * x2[0]")],
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutants_of_the_naive_rule_fail_the_pin(pinned_pairs, name):
    """Plants one mistake in a copy of the replica (on the CPU) and checks the pin sees it."""
    _, good, exact = pinned_pairs
    src = inspect.getsource(naive.classify) + "\n" + inspect.getsource(naive.normal)
    mutated = src
    for a, b in MUTANTS[name]:
        assert a in mutated, a
        mutated = mutated.replace(a, b)
    ns = dict(vars(naive))
    exec(compile(mutated, f"<mutant {name}>", "exec"), ns)
    assert _mismatches(ns["classify"], good, exact) > 0
