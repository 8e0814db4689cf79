"""Butcher tableaus of common explicit Runge-Kutta methods, for
``Chain(..., tableau=...)``. Each entry is (a, b): a is s x s (strictly lower
triangle), b has s weights. The models are autonomous, so the nodes c are not
needed.
"""
from __future__ import annotations

from fractions import Fraction


def _tab(rows, weights):
    s = len(weights)
    a = [[0.0] * s for _ in range(s)]
    for j, row in enumerate(rows, start=1):
        for m, v in enumerate(row):
            a[j][m] = float(Fraction(v))
    return a, [float(Fraction(w)) for w in weights]


# explicit midpoint rule, order 2
MIDPOINT = _tab([["1/2"]], ["0", "1"])
# Heun's method, order 2
HEUN2 = _tab([["1"]], ["1/2", "1/2"])
# Kutta's third-order method
KUTTA3 = _tab([["1/2"], ["-1", "2"]], ["1/6", "2/3", "1/6"])
# strong-stability-preserving third-order method of Shu and Osher
SSPRK3 = _tab([["1"], ["1/4", "1/4"]], ["1/6", "1/6", "2/3"])
# the classical fourth-order method (the dedicated kernels run it faster)
RK4 = _tab([["1/2"], ["0", "1/2"], ["0", "0", "1"]], ["1/6", "1/3", "1/3", "1/6"])
# Kutta's 3/8 rule, order 4
RK4_38 = _tab([["1/3"], ["-1/3", "1"], ["1", "-1", "1"]], ["1/8", "3/8", "3/8", "1/8"])
# Dormand and Prince's fifth-order solution, used at a fixed step (the
# embedded fourth-order estimate and its extra stage are not needed)
DOPRI5 = _tab([["1/5"],
               ["3/40", "9/40"],
               ["44/45", "-56/15", "32/9"],
               ["19372/6561", "-25360/2187", "64448/6561", "-212/729"],
               ["9017/3168", "-355/33", "46732/5247", "49/176", "-5103/18656"]],
              ["35/384", "0", "500/1113", "125/192", "-2187/6784", "11/84"])

ALL = {"midpoint": MIDPOINT, "heun2": HEUN2, "kutta3": KUTTA3, "ssprk3": SSPRK3, "rk4": RK4,
       "rk4_38": RK4_38, "dopri5": DOPRI5}
