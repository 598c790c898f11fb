"""Tersoff parameter tables for the oracle (test infrastructure only).

The paper leaves the parameter values out (Section III: the parameters were
fitted empirically).  The values below are Tersoff's published element sets
(Si(B): Tersoff 1988a; Si(C): Tersoff 1988b; C and the Si-C mixing rules:
Tersoff 1989), in the R/D cutoff parameterisation: Tersoff's own R, S map to
R = (R + S)/2 and D = (S - R)/2.

Table layout: ``table[ti, tj, tk, field]`` with 14 fields in the order
m, gamma, lambda3, c, d, h, n, beta, lambda2, B, R, D, lambda1, A.
Pair quantities of (i, j) live in the entry [ti, tj, tj]; the three-body
quantities of (i, j, k) and the cutoff of the (i, k) distance live in
[ti, tj, tk].

This module is written independently of the product's own table builder;
the tests compare the two.
"""
import math

import numpy as np

FIELDS = ("m", "gamma", "lam3", "c", "d", "h", "n", "beta", "lam2", "B", "R", "D", "lam1", "A")
IDX = {name: i for i, name in enumerate(FIELDS)}

# element sets: (A, B, lam1, lam2, beta, n, c, d, h, lam3, m, gamma, R_tersoff, S_tersoff)
SI_B = dict(A=3264.7, B=95.373, lam1=3.2394, lam2=1.3258, beta=0.33675, n=22.956,
            c=4.8381, d=2.0417, h=0.0, lam3=1.3258, m=3.0, gamma=1.0, Rt=2.8, St=3.2)
SI_C = dict(A=1830.8, B=471.18, lam1=2.4799, lam2=1.7322, beta=1.1e-6, n=0.78734,
            c=1.0039e5, d=16.217, h=-0.59825, lam3=0.0, m=3.0, gamma=1.0, Rt=2.7, St=3.0)
CARBON = dict(A=1393.6, B=346.74, lam1=3.4879, lam2=2.2119, beta=1.5724e-7, n=0.72751,
              c=3.8049e4, d=4.3484, h=-0.57058, lam3=0.0, m=3.0, gamma=1.0, Rt=1.8, St=2.1)
CHI_SIC = 0.9776


def _row(three, pair_a, pair_b, cut_rs):
    """One table entry: three-body fields from `three`, pair fields from the
    (pair_a, pair_b) dicts (already mixed), cutoff from (Rt, St)."""
    r = np.zeros(14)
    r[IDX["m"]] = three["m"]
    r[IDX["gamma"]] = three["gamma"]
    r[IDX["lam3"]] = three["lam3"]
    r[IDX["c"]] = three["c"]
    r[IDX["d"]] = three["d"]
    r[IDX["h"]] = three["h"]
    r[IDX["n"]] = pair_a["n"]
    r[IDX["beta"]] = pair_a["beta"]
    r[IDX["lam2"]] = pair_b["lam2"]
    r[IDX["B"]] = pair_b["B"]
    r[IDX["lam1"]] = pair_b["lam1"]
    r[IDX["A"]] = pair_b["A"]
    Rt, St = cut_rs
    r[IDX["R"]] = 0.5 * (Rt + St)
    r[IDX["D"]] = 0.5 * (St - Rt)
    return r


def single(elem, R=None, D=None):
    """1x1x1 table for one element; R, D override the cutoff if given."""
    t = _row(elem, elem, elem, (elem["Rt"], elem["St"])).reshape(1, 1, 1, 14)
    if R is not None:
        t[0, 0, 0, IDX["R"]] = R
    if D is not None:
        t[0, 0, 0, IDX["D"]] = D
    return t


def mixed_pair(a, b, chi):
    """Tersoff 1989 mixing: geometric A, B (B times chi), arithmetic lambdas,
    geometric R and S."""
    return dict(A=math.sqrt(a["A"] * b["A"]), B=chi * math.sqrt(a["B"] * b["B"]),
                lam1=0.5 * (a["lam1"] + b["lam1"]), lam2=0.5 * (a["lam2"] + b["lam2"]),
                Rt=math.sqrt(a["Rt"] * b["Rt"]), St=math.sqrt(a["St"] * b["St"]))


def sic():
    """2x2x2 table, species 0 = Si (Si(C) set), 1 = C."""
    el = [SI_C, CARBON]
    t = np.zeros((2, 2, 2, 14))
    for i in range(2):
        for j in range(2):
            pj = el[i] if i == j else mixed_pair(el[i], el[j], CHI_SIC)
            for k in range(2):
                pk = el[i] if i == k else mixed_pair(el[i], el[k], 1.0)
                row = _row(el[i], el[i], pj, (pk["Rt"], pk["St"]))
                t[i, j, k] = row
    return t


def max_cutoff(table):
    return float(np.max(table[..., IDX["R"]] + table[..., IDX["D"]]))
