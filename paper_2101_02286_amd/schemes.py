"""Compact schemes of the library's callers: left-hand-side bands and
right-hand-side stencils on a uniform periodic grid x_j = j h, h = 2 pi / n.

A scheme is the pair (bands of A, stencil B) of a compact operator
A f' = B f (Sec. 1 Eq. (1)-(2), App. A.2).  The stencil is returned as
(lo, coefs) with out_j = sum_q coefs[q - lo] f_{j+q}; derivative stencils
have the spacing folded in.  This is set-up data for cb_plan and cb_stencil,
not a step of the solve.

  tri6     sixth-order collocated first derivative: bands [1/3, 1, 1/3] (the
           sixth-order system of Sec. 5), RHS weights a = 14/9, b = 1/9
  penta10  tenth-order collocated first derivative: bands
           [1/20, 1/2, 1, 1/2, 1/20], RHS weights a = 17/12, b = 101/150,
           c = 1/100 (the paper gives no pentadiagonal numbers; these satisfy
           the Taylor order conditions through tenth order)
  interp6  sixth-order interpolation, App. A.2: bands [3/10, 1, 3/10],
           a = 3/2, b = 1/10; "c2s" reads collocated f and returns values at
           x_{j+1/2}, "s2c" reads staggered f (f_k at x_{k+1/2}) and returns
           values at x_j
  stag6    sixth-order staggered first derivative, App. A.2: bands
           [9/62, 1, 9/62], a = 63/62, b = 17/62; "c2s" and "s2c" as above
  hept12   twelfth-order collocated first derivative with a heptadiagonal
           left-hand side (Sec. 2's general band, r = 3): bands
           [1/400, 9/100, 9/16, 1, 9/16, 9/100, 1/400], a = 21/16,
           b = 231/250, c = 147/2000 (the Taylor order conditions through
           twelfth order; symmetric positive definite, not diagonally dominant)
"""
import math

_SCHEMES = {
    # name: (alpha, beta, gamma, a, b, c)
    "tri6": (1.0 / 3.0, 0.0, 0.0, 14.0 / 9.0, 1.0 / 9.0, 0.0),
    "penta10": (1.0 / 2.0, 1.0 / 20.0, 0.0, 17.0 / 12.0, 101.0 / 150.0, 1.0 / 100.0),
    "hept12": (9.0 / 16.0, 9.0 / 100.0, 1.0 / 400.0, 21.0 / 16.0, 231.0 / 250.0, 147.0 / 2000.0),
    "interp6": (3.0 / 10.0, 0.0, 0.0, 3.0 / 2.0, 1.0 / 10.0, 0.0),
    "stag6": (9.0 / 62.0, 0.0, 0.0, 63.0 / 62.0, 17.0 / 62.0, 0.0),
}
DERIVATIVES = ("tri6", "penta10", "hept12")


def bands(name):
    """Constant bands a_{-r..r} of the scheme's left-hand side."""
    al, be, ga = _SCHEMES[name][:3]
    if ga:
        return [ga, be, al, 1.0, al, be, ga]
    return [be, al, 1.0, al, be] if be else [al, 1.0, al]


def spacing(n):
    return 2.0 * math.pi / n


def stencil(name, n, grid="c2s"):
    """(lo, coefs) of the scheme's periodic right-hand side for lines of n points.

    Collocated derivatives (tri6, penta10) ignore `grid`."""
    al, be, ga, a, b, c = _SCHEMES[name]
    h = spacing(n)
    if name in DERIVATIVES:
        if c:
            return -3, [-c / (6 * h), -b / (4 * h), -a / (2 * h), 0.0, a / (2 * h), b / (4 * h), c / (6 * h)]
        return -2, [-b / (4 * h), -a / (2 * h), 0.0, a / (2 * h), b / (4 * h)]
    # staggered pairs: the four neighbours at half-integer distances
    # -3h/2, -h/2, h/2, 3h/2 from the output point
    lo = -1 if grid == "c2s" else -2
    if grid not in ("c2s", "s2c"):
        raise ValueError("grid must be 'c2s' or 's2c'")
    if name == "interp6":
        return lo, [b / 2, a / 2, a / 2, b / 2]
    if name == "stag6":
        return lo, [-b / (3 * h), -a / h, a / h, b / (3 * h)]
    raise ValueError(name)
