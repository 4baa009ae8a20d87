"""Free-energy differences by the Bennett acceptance ratio (nnp_bar, host
code of the library), for reweighting stored snapshots with the network's
energies (energy-only evaluation, no forces).

Energies are in kcal/mol; beta = 1 / (k_B T).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _native as nat

KB_KCAL = 0.0019872042586408316  # Boltzmann constant, kcal/mol/K


def beta_at(temperature_k: float) -> float:
    return 1.0 / (KB_KCAL * temperature_k)


def bar_reduced(u, v, lw0=None, lw1=None):
    """beta (F_1 - F_0) and its asymptotic standard deviation from reduced
    differences: u = beta (U_1 - U_0) on samples of state 0, v = beta (U_0 -
    U_1) on samples of state 1, optional log weights of the samples."""
    arr = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64)
    u, v, lw0, lw1 = arr(u), arr(v), arr(lw0), arr(lw1)
    if lw0 is not None and lw0.shape != u.shape:
        raise ValueError("lw0 must match u")
    if lw1 is not None and lw1.shape != v.shape:
        raise ValueError("lw1 must match v")
    p = lambda a: None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))
    d, s = C.c_double(), C.c_double()
    nat.check(nat.load().nnp_bar(len(u), p(u), p(lw0), len(v), p(v), p(lw1), C.byref(d), C.byref(s)))
    return d.value, s.value


def bar(U0_on_0, U1_on_0, U0_on_1, U1_on_1, beta: float):
    """F_1 - F_0 (energy units) and its standard deviation from the two
    states' energies evaluated on samples of state 0 and of state 1."""
    u = beta * (np.asarray(U1_on_0, np.float64) - np.asarray(U0_on_0, np.float64))
    v = beta * (np.asarray(U0_on_1, np.float64) - np.asarray(U1_on_1, np.float64))
    d, s = bar_reduced(u, v)
    return d / beta, s / beta


def bar_reweighted(U0_on_0, U1_on_0, U0_on_1, U1_on_1, Ut0_on_0, Ut1_on_0, Ut0_on_1, Ut1_on_1,
                   beta: float):
    """F'_1 - F'_0 of a target potential U' (energies Ut*) from samples of a
    reference ensemble U (energies U*): each sample of state s is weighted by
    exp(-beta (U'_s - U_s)) and the BAR equation is solved with the target's
    energy differences."""
    f = lambda a: np.asarray(a, np.float64)
    u = beta * (f(Ut1_on_0) - f(Ut0_on_0))
    v = beta * (f(Ut0_on_1) - f(Ut1_on_1))
    lw0 = -beta * (f(Ut0_on_0) - f(U0_on_0))
    lw1 = -beta * (f(Ut1_on_1) - f(U1_on_1))
    d, s = bar_reduced(u, v, lw0, lw1)
    return d / beta, s / beta
