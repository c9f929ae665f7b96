"""Exact-rational derivation of the FAM reconstruction operators.

Test infrastructure: part of the FP64 CPU oracle (see ``oracle/__init__.py``).

Everything here follows the *definitions* in Sec. 2.4 of the paper (compact linear
reconstructions and consistency), not the printed coefficient and jump tables of
the appendices.  The printed tables are used only by the tests, as pins against
which the solutions computed here are checked.

Coordinates are cell-local and scaled: xi = (x - x_i)/dx, eta = (y - y_j)/dy, so
every cell is the unit square (unit interval in 1D) and the neighbour at offset
(a, b) is [a-1/2, a+1/2] x [b-1/2, b+1/2].  A polynomial is a dict mapping a
monomial exponent tuple to a Fraction coefficient.

* 1D, eq. (5): cubic Q matching the averages of cells i-1, i, i+1 and the first
  moment of cell i.  eq. (6): quintic Q matching averages and first moments of
  cells i-1, i, i+1.  p_2 = Pi_2 Q (FAM3), p_3 = Q (FAM4), p_4 = Pi_4 Q (FAM5),
  p_5 = Q (FAM6).
* 2D, system (Qxy_quartic): 11 constraints (nine averages of the 3x3 patch, both
  first moments of the centre) in the space P_3 + span{xi^2 eta^2}, which is the
  span of the first 11 basis functions of the appendix on 2D orthogonal bases.  p_3 = Pi_2 Q, p_4 = Pi_3 Q.
* 2D, system (Qxy_quintic): 23 constraints (nine averages, x-moments of patch
  cells {1,3,4,5,6,7,9}, y-moments of {1,2,3,5,7,8,9}) in P_5 + span{xi^4 eta^2,
  xi^2 eta^4} (the span of all 23 basis functions of that appendix).  p_5 = Pi_4 Q,
  p_6 = Pi_5 Q.
* Pi_m is the L2(cell) orthogonal projection onto complete polynomials of total
  degree <= m, computed here from Gram matrices (not by truncating an
  orthogonal expansion).

Patch numbering (Sec. 2.4): I_1=(i-1,j-1), I_2=(i,j-1), I_3=(i+1,j-1), I_4=(i-1,j),
I_5=(i,j), I_6=(i+1,j), I_7=(i-1,j+1), I_8=(i,j+1), I_9=(i+1,j+1).
"""
from fractions import Fraction as Fr
from functools import lru_cache

HALF = Fr(1, 2)


# ----------------------------------------------------------------------------
# exact linear algebra
# ----------------------------------------------------------------------------
def solve_exact(A, B):
    """Solve A X = B exactly (Gauss-Jordan with Fractions). A: n x n, B: n x m."""
    n = len(A)
    M = [list(map(Fr, A[r])) + list(map(Fr, B[r])) for r in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        p = M[col][col]
        M[col] = [v / p for v in M[col]]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col]
                M[r] = [a - f * b for a, b in zip(M[r], M[col])]
    return [row[n:] for row in M]


def det_exact(A):
    n = len(A)
    M = [list(map(Fr, row)) for row in A]
    det = Fr(1)
    for col in range(n):
        piv = next((r for r in range(col, n) if M[r][col] != 0), None)
        if piv is None:
            return Fr(0)
        if piv != col:
            M[col], M[piv] = M[piv], M[col]
            det = -det
        det *= M[col][col]
        for r in range(col + 1, n):
            f = M[r][col] / M[col][col]
            M[r] = [a - f * b for a, b in zip(M[r], M[col])]
    return det


def matmul_exact(A, B):
    return [[sum((A[i][k] * B[k][j] for k in range(len(B))), Fr(0))
             for j in range(len(B[0]))] for i in range(len(A))]


# ----------------------------------------------------------------------------
# monomial integrals on shifted unit cells
# ----------------------------------------------------------------------------
def int_1d(p, a):
    """Integral of t^p over the unit cell [a-1/2, a+1/2]."""
    lo, hi = Fr(a) - HALF, Fr(a) + HALF
    return (hi ** (p + 1) - lo ** (p + 1)) / (p + 1)


def moment_1d(p, a, kind):
    """Scaled moment of t^p over cell a: kind 0 -> average, kind 1 -> against (t - a)."""
    if kind == 0:
        return int_1d(p, a)
    return int_1d(p + 1, a) - a * int_1d(p, a)


def moment_2d(mono, a, b, kind):
    """Scaled moment of xi^p eta^q over cell (a, b).

    kind 0: average; kind 1: against (xi - a); kind 2: against (eta - b).
    """
    p, q = mono
    if kind == 0:
        return int_1d(p, a) * int_1d(q, b)
    if kind == 1:
        return moment_1d(p, a, 1) * int_1d(q, b)
    return int_1d(p, a) * moment_1d(q, b, 1)


# ----------------------------------------------------------------------------
# spaces and constraint lists
# ----------------------------------------------------------------------------
def complete_1d(deg):
    return [(p,) for p in range(deg + 1)]


def complete_2d(deg):
    return [(p, t - p) for t in range(deg + 1) for p in range(t, -1, -1)]


PATCH_OFFSETS = {l: ((l - 1) % 3 - 1, (l - 1) // 3 - 1) for l in range(1, 10)}


def space_1d(k):
    """Monomials spanning the auxiliary Q of eq. (5) (k=3,4) or eq. (6) (k=5,6)."""
    return complete_1d(3 if k in (3, 4) else 5)


def constraints_1d(k):
    """(cell offset, kind) list; the order defines the stencil input vector."""
    if k in (3, 4):
        return [(-1, 0), (0, 0), (1, 0), (0, 1)]
    return [(-1, 0), (0, 0), (1, 0), (-1, 1), (0, 1), (1, 1)]


def proj_degree_1d(k):
    return k - 1


def space_2d(k):
    if k in (3, 4):
        return complete_2d(3) + [(2, 2)]
    return complete_2d(5) + [(4, 2), (2, 4)]


def constraints_2d(k):
    """(patch index l, kind) list in the order of the moment system."""
    cons = [(l, 0) for l in range(1, 10)]
    if k in (3, 4):
        cons += [(5, 1), (5, 2)]
    else:
        cons += [(l, 1) for l in (1, 3, 4, 5, 6, 7, 9)]
        cons += [(l, 2) for l in (1, 2, 3, 5, 7, 8, 9)]
    return cons


def proj_degree_2d(k):
    return k - 1


# ----------------------------------------------------------------------------
# reconstruction operators
# ----------------------------------------------------------------------------
def _gram(rows, cols, dim):
    if dim == 1:
        return [[int_1d(r[0] + c[0], 0) for c in cols] for r in rows]
    return [[int_1d(r[0] + c[0], 0) * int_1d(r[1] + c[1], 0) for c in cols] for r in rows]


@lru_cache(maxsize=None)
def system_matrix(dim, k):
    """Moment-matching matrix A: rows = constraints, cols = auxiliary-space monomials."""
    if dim == 1:
        return [[moment_1d(m[0], a, kind) for m in space_1d(k)] for a, kind in constraints_1d(k)]
    rows = []
    for l, kind in constraints_2d(k):
        a, b = PATCH_OFFSETS[l]
        rows.append([moment_2d(m, a, b, kind) for m in space_2d(k)])
    return rows


@lru_cache(maxsize=None)
def aux_operator(dim, k):
    """Exact map stencil moments -> monomial coefficients of the auxiliary Q."""
    A = system_matrix(dim, k)
    n = len(A)
    eye = [[Fr(int(r == c)) for c in range(n)] for r in range(n)]
    return solve_exact(A, eye)


@lru_cache(maxsize=None)
def projection(dim, k):
    """Exact L2(cell) projection matrix from the auxiliary space onto P_{k-1}."""
    space = space_1d(k) if dim == 1 else space_2d(k)
    target = complete_1d(k - 1) if dim == 1 else complete_2d(k - 1)
    G_tt = _gram(target, target, dim)
    G_ts = _gram(target, space, dim)
    return solve_exact(G_tt, G_ts)


@lru_cache(maxsize=None)
def recon_operator(dim, k):
    """Exact map stencil moments -> monomial coefficients of p_k (degree k-1).

    Returns (monomials, matrix) with matrix[row=monomial][col=stencil input].
    """
    target = complete_1d(k - 1) if dim == 1 else complete_2d(k - 1)
    return target, matmul_exact(projection(dim, k), aux_operator(dim, k))


def eval_poly(monos, coeffs, pt):
    """Evaluate sum_c coeffs[c] * pt^monos[c] exactly."""
    total = Fr(0)
    for m, c in zip(monos, coeffs):
        term = Fr(c)
        for e, x in zip(m, pt):
            term *= Fr(x) ** e
        total += term
    return total


def stencil_moments_of_poly_1d(k, monos, coeffs):
    """Exact stencil input vector (constraint order) of a 1D polynomial."""
    return [sum((Fr(c) * moment_1d(m[0], a, kind) for m, c in zip(monos, coeffs)), Fr(0))
            for a, kind in constraints_1d(k)]


def stencil_moments_of_poly_2d(k, monos, coeffs, centre=(0, 0)):
    """Exact stencil input vector of a 2D polynomial, patch centred at `centre`."""
    out = []
    for l, kind in constraints_2d(k):
        a, b = PATCH_OFFSETS[l]
        a += centre[0]
        b += centre[1]
        out.append(sum((Fr(c) * moment_2d(m, a, b, kind) for m, c in zip(monos, coeffs)), Fr(0)))
    return out


# ----------------------------------------------------------------------------
# derived linear forms used as pins (jumps at interfaces)
# ----------------------------------------------------------------------------
def jump_forms_1d(k):
    """Interface jump [[u]]_{i+1/2} = p_{i+1}(-1/2) - p_i(1/2) as exact linear forms.

    Returns dicts {(cell offset s, moment r): coefficient} with s in -1..2.
    """
    monos, R = recon_operator(1, k)
    cons = constraints_1d(k)
    out = {}
    for owner, side, sign in ((0, HALF, -1), (1, -HALF, +1)):
        vals = [eval_poly(monos, [R[m][c] for m in range(len(monos))], (side,)) for c in range(len(cons))]
        for (a, kind), v in zip(cons, vals):
            key = (owner + a, kind)
            out[key] = out.get(key, Fr(0)) + sign * v
    return {k_: v for k_, v in out.items() if v != 0}


def jump_matrices_2d(k, use_full_aux=False):
    """A_k, B_k, C_k (4x3, rows s=-1..2, cols l=-1..1) of the x-interface jump.

    [[u]]_{i+1/2,j} = p_{i+1,j}(-1/2, 0) - p_{i,j}(1/2, 0) written as Frobenius
    products with the 4x3 blocks [u^{(r)}_{i+s, j+l}], r = 0, 1, 2 (eq. 2Djump).
    With use_full_aux=True the auxiliary Q is used in place of the projected p_k.
    """
    if use_full_aux:
        monos, R = space_2d(k), aux_operator(2, k)
    else:
        monos, R = recon_operator(2, k)
    cons = constraints_2d(k)
    mats = [[[Fr(0)] * 3 for _ in range(4)] for _ in range(3)]
    for owner, side, sign in ((0, HALF, -1), (1, -HALF, +1)):
        for c, (l, kind) in enumerate(cons):
            v = eval_poly(monos, [R[m][c] for m in range(len(monos))], (side, 0))
            a, b = PATCH_OFFSETS[l]
            s = owner + a
            mats[kind][s + 1][b + 1] += sign * v
    return mats
