"""The alternative point formulas, compiled for the CPU, against the oracle's replicas.

Each formula's two circle points equal oracle/ablation.py's binary64 replica bit for bit,
and the formula reports points exactly where the replica does (the replica's own pins live
in tests/test_oracle_ablation.py).
"""

import ctypes
import math

import numpy as np
import pytest

from oracle import ablation as AB, geometry as G
from paper_2510_09892_amd import inputs

import test_hostcheck as TH

FORMULAS = {"eq22": 0, "eq21": 1, "eq71": 2, "kahan": 3}


@pytest.fixture(scope="module")
def hc():
    lib = ctypes.CDLL(TH.LIBPATH)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    lib.sphint_hostcheck_circle.argtypes = [ctypes.c_int, ctypes.c_int64] + [dp] * 9 + [ip]
    return lib


def run_circle(hc, formula, soa):
    soa = [np.ascontiguousarray(a, dtype=np.float64) for a in soa]
    n = len(soa[0])
    ox, oy = np.zeros(2 * n), np.zeros(2 * n)
    ok = np.zeros(n, np.int32)
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    hc.sphint_hostcheck_circle(formula, n, *[dp(a) for a in soa], dp(ox), dp(oy),
                               ok.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return ox.reshape(-1, 2), oy.reshape(-1, 2), ok


def compare_with_replica(name, soa, ox, oy, ok):
    n = len(soa[0])
    for i in range(n):
        x1 = (float(soa[0][i]), float(soa[1][i]), float(soa[2][i]))
        x2 = (float(soa[3][i]), float(soa[4][i]), float(soa[5][i]))
        z0 = float(soa[6][i])
        pp = AB.point(name, x1, x2, z0, G.PLUS)
        pm = AB.point(name, x1, x2, z0, G.MINUS)
        assert bool(ok[i]) == (pp is not None), (name, i)
        if pp is None:
            assert ox[i, 0] == oy[i, 0] == ox[i, 1] == oy[i, 1] == 0.0
            continue
        assert (ox[i, 0], oy[i, 0]) == pp, (name, i)
        assert (ox[i, 1], oy[i, 1]) == pm, (name, i)


def workloads():
    rows = [inputs.uniform_arcs(1500, seed_tag=55).soa(), inputs.ill_conditioned(1500, seed_tag=56).soa()]
    special = np.array([
        (1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0),        # equator: n^z = 1
        (1.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.5),        # meridian
        (1.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0),        # zero normal
        (1.0, 0.0, 0.0, 0.0, 1.0, 1e-9, 0.0),       # great circle 1e-9 from the equator
        (0.6, 0.8, 0.0, 0.0, 0.6, 0.8, 0.99),       # beyond the top
        (2.0, 0.0, 0.0, 0.0, 3.0, 3.0, -0.25),      # unnormalised endpoints
    ])
    rows.append([special[:, k].copy() for k in range(7)])
    return rows


@pytest.mark.parametrize("name", list(FORMULAS))
def test_formula_equals_replica(hc, name):
    for soa in workloads():
        ox, oy, ok = run_circle(hc, FORMULAS[name], soa)
        compare_with_replica(name, soa, ox, oy, ok)
