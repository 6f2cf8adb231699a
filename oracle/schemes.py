"""Compact-scheme coefficients for the oracle (test infrastructure only).

Each scheme is the pair (left-hand-side bands, right-hand-side stencil) of a
compact finite-difference operator on a uniform periodic grid x_j = j*h,
h = 2*pi/n.  The oracle keeps its own copy of these numbers; the HIP library
receives bands and stencils as plain arguments and shares nothing with this
file.

Stencils are (lo, coefs): out_j = sum_{q=lo}^{lo+len-1} coefs[q-lo] * f_{j+q}.
"""
from fractions import Fraction as Fr

# Sec. 1 Eq. (1), with the sixth-order choice of Sec. 5 (bands [1/3, 1, 1/3]):
# alpha f'_{j-1} + f'_j + alpha f'_{j+1} = a (f_{j+1}-f_{j-1})/(2h) + b (f_{j+2}-f_{j-2})/(4h)
DERIV6 = dict(alpha=Fr(1, 3), beta=Fr(0), a=Fr(14, 9), b=Fr(1, 9), c=Fr(0))

# Tenth-order member of the same collocated family (pentadiagonal; Sec. 2
# treats penta-diagonal systems, Eq. (6)).  The paper gives no numbers for it;
# these are the ones fixed by the Taylor-series order conditions, checked
# exactly in the tests.
DERIV10 = dict(alpha=Fr(1, 2), beta=Fr(1, 20), a=Fr(17, 12), b=Fr(101, 150), c=Fr(1, 100))

# Twelfth-order member with three left-hand neighbours (heptadiagonal, the
# general band of Sec. 2 Eq. (4) with r = 3):
# gamma f'_{j-3} + beta f'_{j-2} + alpha f'_{j-1} + f'_j + ... (symmetric)
#   = a (f_{j+1}-f_{j-1})/(2h) + b (f_{j+2}-f_{j-2})/(4h) + c (f_{j+3}-f_{j-3})/(6h).
# The six coefficients are the unique solution of the Taylor order
# conditions through twelfth order (checked exactly in the tests); the
# matrix is not diagonally dominant but its symbol stays positive (>= 1/20),
# so it is symmetric positive definite.
DERIV12H = dict(alpha=Fr(9, 16), beta=Fr(9, 100), gamma=Fr(1, 400), a=Fr(21, 16), b=Fr(231, 250),
                c=Fr(147, 2000))

# Sec. 1 Eq. (2) and App. A.2: collocated -> staggered interpolation,
# alpha^ f^I_{j-1} + f^I_j + alpha^ f^I_{j+1} = a (f_{j+1/2}+f_{j-1/2})/2 + b (f_{j+3/2}+f_{j-3/2})/2
INTERP6 = dict(alpha=Fr(3, 10), a=Fr(3, 2), b=Fr(1, 10))

# App. A.2: staggered sixth-order first derivative,
# (9/62) f'_{j-1} + f'_j + (9/62) f'_{j+1} = (63/62)(f_{j+1/2}-f_{j-1/2})/D + (17/62)(f_{j+3/2}-f_{j-3/2})/(3D)
STAG6 = dict(alpha=Fr(9, 62), a=Fr(63, 62), b=Fr(17, 62))


def bands_collocated(s):
    """LHS bands [gamma, beta, alpha, 1, alpha, beta, gamma] (r=3),
    [beta, alpha, 1, alpha, beta] (r=2) or [alpha, 1, alpha] (r=1)."""
    al, be, ga = float(s["alpha"]), float(s.get("beta", 0)), float(s.get("gamma", 0))
    if ga != 0.0:
        return [ga, be, al, 1.0, al, be, ga]
    if be != 0.0:
        return [be, al, 1.0, al, be]
    return [al, 1.0, al]


def stencil_deriv_collocated(s, h):
    """f'_j at x_j from f at x_{j+q}: antisymmetric 7-point (or 5-point) stencil."""
    a, b, c = float(s["a"]), float(s["b"]), float(s["c"])
    if c != 0.0:
        return -3, [-c / (6 * h), -b / (4 * h), -a / (2 * h), 0.0, a / (2 * h), b / (4 * h), c / (6 * h)]
    return -2, [-b / (4 * h), -a / (2 * h), 0.0, a / (2 * h), b / (4 * h)]


def stencil_interp_c2s(s):
    """f^I_j at x_{j+1/2} from collocated f: uses f_{j-1}, f_j, f_{j+1}, f_{j+2}."""
    a, b = float(s["a"]), float(s["b"])
    return -1, [b / 2, a / 2, a / 2, b / 2]


def stencil_interp_s2c(s):
    """f^I_j at x_j from staggered f^s_k (at x_{k+1/2}): uses f^s_{j-2..j+1}."""
    a, b = float(s["a"]), float(s["b"])
    return -2, [b / 2, a / 2, a / 2, b / 2]


def stencil_deriv_c2s(s, h):
    """f'_j at x_{j+1/2} from collocated f_{j-1..j+2} (App. A.2 read on the staggered grid)."""
    a, b = float(s["a"]), float(s["b"])
    return -1, [-b / (3 * h), -a / h, a / h, b / (3 * h)]


def stencil_deriv_s2c(s, h):
    """f'_j at x_j from staggered f^s_{j-2..j+1} (f^s_k sits at x_{k+1/2})."""
    a, b = float(s["a"]), float(s["b"])
    return -2, [-b / (3 * h), -a / h, a / h, b / (3 * h)]
