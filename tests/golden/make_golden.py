"""Write the golden trajectories of tiny TV-MD and FA-MD problems.

These fixtures pin the FP64 oracle to a computation that shares none of its
code and none of its arithmetic route. Here every operator is an explicit
dense matrix built from its definition, and every z-step is a dense linear
solve. No FFT, no diagonalisation, and no Parseval identity is assumed.
FA-MD runs in exact rational arithmetic. Its steps, the Haar filters
included, are rational on any grid. TV-MD needs the square root of the vector
soft threshold, so it runs in 60-digit decimal arithmetic.

Steps, in the paper's order (Almeida & Figueiredo, Sec. IV):

* z-step of Alg. 2 / Alg. 3, written as the normal equations it solves:
      (mu1 A^T A + mu2 R^T R) z = mu1 A^T zeta1 + mu2 R^T zeta2
  with R = (D^h; D^v) for TV (eq. (33)) and R = P for FA (eqs. (24)-(25));
* data step (the mask prox of eq. (40), used as eq. (49) in TV-MD):
  u1 = (M^T y + mu1 (A z - d1)) / (m + mu1),
  d1 <- d1 - (A z - u1);
* regulariser step: vector soft threshold of (D z - d_TV) by lambda / mu2
  (TV, Sec. III-C), component-wise soft threshold of (P z - d2) by
  lambda / mu2 (FA, eq. (16)); d <- d - (R z - u).

Conventions (the same readings the oracle states):
* A is periodic convolution, (A x)[r, c] = sum h[a+l, b+l] x[r-a, c-b];
* D^h, D^v are periodic forward differences;
* P is the undecimated Haar frame, levels j = 1..J at dilation 2^(j-1),
  filters (x[i] + x[i+s]) / 2 and (x[i] - x[i+s]) / 2 on each axis.
  The z-trajectory does not depend on the band order or on the filter
  direction (either one permutes, shifts or negates whole bands, which the
  soft threshold and P^T undo).

Inputs are dyadic rationals, so that the FP64 oracle receives them exactly.

At every recorded iteration k >= 2 the files also hold the primal and dual
residuals of the stopping rule (definitions in ``residuals``), from the same
exact state: u_k, u_{k-1}, d_k and G z_k.

The FS fixture (method fs) runs FS-MD, the frame-synthesis formulation of
eq. (35): unknowns are the 3J+1 coefficient bands z of the image x = W z with
W = P^T, H1 = A W, H2 = I, the z-step as the dense solve of its normal
equations (mu1 W^T A^T A W + mu2 I) z = mu1 W^T A^T zeta1 + mu2 zeta2 (no
use of eq. (18)), the data prox of eq. (40) on A W z and the soft threshold of
eq. (16) on z. Its "z" lines hold the image x_k = W z_k; its residuals take
the blocks A W z - u1 and z - u2, and its objective is eq. (35).

The CG fixtures (method cg) run the Reeves-Sorel variants on the same tiny
problems: H1 = M A, the z-step through C = (A^T A + gamma R^T R)^{-1} (a dense
solve) and the boundary system S v = v - B C B^T v with B the rows of A at the
unobserved pixels, one conjugate-gradient (steepest-descent) step per
iteration from the previous v (Sec. IV-B..IV-D). The data block of their
residuals is M A z - u1.

Run ``python tests/golden/make_golden.py`` to rewrite the ``.txt`` files.
"""

import os
from decimal import Decimal, getcontext
from fractions import Fraction as Q

HERE = os.path.dirname(os.path.abspath(__file__))
getcontext().prec = 60


# ----------------------------------------------------------------- problems
# Each problem: grid H x W, kernel (odd side, dyadic taps summing to 1),
# mask (0/1, row-major), y (dyadic, row-major), lambda, mu1, mu2, iterations.

def _tv_problem():
    H, W = 5, 6
    h = [[0, 1, 0],
         [2, 5, 1],
         [0, 3, 4]]                                      # sum 16; asymmetric
    h = [[Q(v, 16) for v in row] for row in h]
    mask = [1, 1, 0, 1, 1, 1,
            1, 0, 1, 1, 1, 0,
            1, 1, 1, 1, 0, 1,
            0, 1, 1, 1, 1, 1,
            1, 1, 1, 0, 1, 1]
    yv = [3, 7, 0, 5, 6, 2,
          4, 0, 8, 1, 7, 0,
          2, 6, 3, 8, 0, 5,
          0, 1, 7, 4, 2, 6,
          5, 3, 1, 0, 8, 4]
    y = [Q(v, 8) for v in yv]
    return dict(name="tv_md_5x6", reg="tv", H=H, W=W, kernel=h, mask=mask, y=y,
                lam=Q(1, 64), mu1=Q(1, 2), mu2=Q(1, 4), iters=8, record=[1, 2, 3, 5, 8])


def _fa_problem():
    H, W = 4, 6
    h = [[1, 0, 2],
         [0, 6, 3],
         [1, 2, 1]]                                      # sum 16; asymmetric
    h = [[Q(v, 16) for v in row] for row in h]
    mask = [1, 1, 1, 0, 1, 1,
            1, 0, 1, 1, 1, 1,
            1, 1, 1, 1, 0, 1,
            0, 1, 1, 1, 1, 1]
    yv = [6, 1, 4, 0, 7, 3,
          2, 0, 5, 8, 1, 6,
          7, 3, 0, 2, 0, 4,
          0, 5, 6, 1, 3, 8]
    y = [Q(v, 8) for v in yv]
    return dict(name="fa_md_4x6_J2", reg="fa", J=2, H=H, W=W, kernel=h, mask=mask, y=y,
                lam=Q(1, 32), mu1=Q(1, 2), mu2=Q(1, 4), iters=8, record=[1, 2, 3, 5, 8])


def _grid(H, W, seed, top):
    """Deterministic small integers in [0, top] from a linear congruential sequence."""
    v, out = seed, []
    for _ in range(H * W):
        v = (1103515245 * v + 12345) % (1 << 31)
        out.append((v >> 16) % (top + 1))
    return out


def _tv_problem_8x10():
    H, W = 8, 10
    h = [[0, 1, 1, 0, 0],
         [1, 2, 3, 1, 0],
         [0, 3, 30, 4, 1],
         [0, 1, 4, 2, 0],
         [1, 0, 1, 1, 7]]                                # sum 64; asymmetric
    h = [[Q(v, 64) for v in row] for row in h]
    mask = [0 if v == 0 else 1 for v in _grid(H, W, 11, 4)]
    y = [Q(v, 16) * m for v, m in zip(_grid(H, W, 12, 16), mask)]
    return dict(name="tv_md_8x10", reg="tv", H=H, W=W, kernel=h, mask=mask, y=y,
                lam=Q(1, 128), mu1=Q(1, 4), mu2=Q(1, 8), iters=8, record=[1, 2, 3, 5, 8])


def _fa_problem_8x8():
    H, W = 8, 8
    h = [[1, 2, 0],
         [0, 8, 3],
         [1, 0, 1]]                                      # sum 16; asymmetric
    h = [[Q(v, 16) for v in row] for row in h]
    mask = [0 if v == 0 else 1 for v in _grid(H, W, 21, 4)]
    y = [Q(v, 16) * m for v, m in zip(_grid(H, W, 22, 16), mask)]
    return dict(name="fa_md_8x8_J3", reg="fa", J=3, H=H, W=W, kernel=h, mask=mask, y=y,
                lam=Q(1, 64), mu1=Q(1, 2), mu2=Q(1, 8), iters=8, record=[1, 2, 3, 5, 8])


def _tv_cg_problem():
    # TV-CG (Sec. IV-D, Reeves-Sorel) on the 5 x 6 TV-MD problem
    return dict(_tv_problem(), name="tv_cg_5x6", method="cg")


def _fa_cg_problem():
    # FA-CG (Sec. IV-C, Reeves-Sorel) on the 4 x 6 FA-MD problem
    return dict(_fa_problem(), name="fa_cg_4x6_J2", method="cg")


def _fs_problem():
    # FS-MD (Sec. IV-C, frame synthesis) on the 4 x 6 FA-MD problem's data
    return dict(_fa_problem(), name="fs_md_4x6_J2", method="fs")


PROBLEMS = (_tv_problem, _fa_problem, _tv_problem_8x10, _fa_problem_8x8, _tv_cg_problem, _fa_cg_problem,
            _fs_problem)


# ----------------------------------------------------------------- dense algebra

def zeros(n, m, zero):
    return [[zero] * m for _ in range(n)]


def matvec(M, x):
    return [sum((a * b for a, b in zip(row, x)), x[0] * 0) for row in M]


def transpose(M):
    return [list(col) for col in zip(*M)]


def matmul(A, B):
    Bt = transpose(B)
    return [[sum((a * b for a, b in zip(row, col)), row[0] * 0) for col in Bt] for row in A]


def add(*vs):
    return [sum(t[1:], t[0]) for t in zip(*vs)]


def scale(s, v):
    return [s * a for a in v]


def lu_factor(M):
    """Gaussian elimination with partial pivoting: (rows of U, multipliers, pivot order).

    Exact for Fractions; the z-step matrix is factored once per problem.
    """
    n = len(M)
    U = [list(r) for r in M]
    perm = list(range(n))
    L = [[None] * n for _ in range(n)]
    for k in range(n):
        p = max(range(k, n), key=lambda i: abs(U[i][k]))
        if U[p][k] == 0:
            raise ZeroDivisionError("singular system")
        U[k], U[p] = U[p], U[k]
        L[k], L[p] = L[p], L[k]
        perm[k], perm[p] = perm[p], perm[k]
        for i in range(k + 1, n):
            f = U[i][k] / U[k][k]
            L[i][k] = f
            if f != 0:
                U[i] = [a - f * c for a, c in zip(U[i], U[k])]
    return U, L, perm


def lu_solve(fac, b):
    U, L, perm = fac
    n = len(U)
    x = [b[perm[i]] for i in range(n)]
    for i in range(n):
        for k in range(i):
            if L[i][k]:
                x[i] = x[i] - L[i][k] * x[k]
    for i in range(n - 1, -1, -1):
        s = x[i]
        for j in range(i + 1, n):
            if U[i][j]:
                s = s - U[i][j] * x[j]
        x[i] = s / U[i][i]
    return x


# ----------------------------------------------------------------- operators as matrices

def conv_matrix(h, H, W, one):
    n, k = H * W, len(h)
    l = k // 2
    A = zeros(n, n, one * 0)
    for r in range(H):
        for c in range(W):
            for a in range(-l, l + 1):
                for b in range(-l, l + 1):
                    q = ((r - a) % H) * W + (c - b) % W
                    A[r * W + c][q] += one * h[a + l][b + l]
    return A


def diff_matrices(H, W, one):
    n = H * W
    Dh, Dv = zeros(n, n, one * 0), zeros(n, n, one * 0)
    for r in range(H):
        for c in range(W):
            p = r * W + c
            Dh[p][r * W + (c + 1) % W] += one
            Dh[p][p] -= one
            Dv[p][((r + 1) % H) * W + c] += one
            Dv[p][p] -= one
    return Dh, Dv


def haar_bands(H, W, J, one):
    """The 3J + 1 band matrices of the undecimated Haar frame (each n x n)."""
    half = one / 2

    def axis_op(N, s, sign):
        M = zeros(N, N, one * 0)
        for i in range(N):
            M[i][i] += half
            M[i][(i + s) % N] += sign * half
        return M

    def vert(op):    # acts along rows index r
        n = H * W
        M = zeros(n, n, one * 0)
        for r in range(H):
            for rr in range(H):
                if op[r][rr] != 0:
                    for c in range(W):
                        M[r * W + c][rr * W + c] += op[r][rr]
        return M

    def horz(op):    # acts along column index c
        n = H * W
        M = zeros(n, n, one * 0)
        for r in range(H):
            for c in range(W):
                for cc in range(W):
                    if op[c][cc] != 0:
                        M[r * W + c][r * W + cc] += op[c][cc]
        return M

    n = H * W
    a = [[one if i == j else one * 0 for j in range(n)] for i in range(n)]
    bands = []
    for j in range(1, J + 1):
        s = 2 ** (j - 1)
        Lv, Hv = vert(axis_op(H, s, 1)), vert(axis_op(H, s, -1))
        Lh, Hh = horz(axis_op(W, s, 1)), horz(axis_op(W, s, -1))
        lv, hv = matmul(Lv, a), matmul(Hv, a)
        bands += [matmul(Hh, lv), matmul(Lh, hv), matmul(Hh, hv)]
        a = matmul(Lh, lv)
    bands.append(a)
    return bands


# ----------------------------------------------------------------- the iterations

def _sq(vs):
    return sum((v * v for v in vs), vs[0] * 0)


def _sqrt(v):
    """Square root in 60-digit decimal arithmetic (exact inputs are converted first)."""
    if isinstance(v, Q):
        v = Decimal(v.numerator) / Decimal(v.denominator)
    return v.sqrt() if v > 0 else Decimal(0)


def residuals(Az, Rz, u1, ur, d1, dr, u1_prev, ur_prev, mu1, mu2):
    """Primal and dual residuals of a check iteration, from their definitions.

    With G the stacked operator (A over the regulariser's blocks) and
    Upsilon = diag(mu1 on the data block, mu2 on every regulariser block):
        r_pri  = ||G z - u|| / max(||G z||, ||u||)
        r_dual = ||Upsilon (u_k - u_{k-1})|| / ||Upsilon d_k||
    (the stopping rule is not the paper's, which stops on the relative change
    of the objective in Sec. V; these are the readings the oracle takes).
    """
    pri2 = _sq([a - u for a, u in zip(Az, u1)])
    gz2 = _sq(Az)
    un2 = _sq(u1)
    du2 = _sq([a - b for a, b in zip(u1, u1_prev)])
    dn2 = _sq(d1)
    reg = {"pri": pri2 * 0, "gz": pri2 * 0, "un": pri2 * 0, "du": pri2 * 0, "dn": pri2 * 0}
    for Rb, ub, db, pb_ in zip(Rz, ur, dr, ur_prev):
        reg["pri"] += _sq([a - u for a, u in zip(Rb, ub)])
        reg["gz"] += _sq(Rb)
        reg["un"] += _sq(ub)
        reg["du"] += _sq([a - b for a, b in zip(ub, pb_)])
        reg["dn"] += _sq(db)
    pri = _sqrt(pri2 + reg["pri"])
    den = max(_sqrt(gz2 + reg["gz"]), _sqrt(un2 + reg["un"]))
    dual = _sqrt(mu1 * mu1 * du2 + mu2 * mu2 * reg["du"])
    dden = _sqrt(mu1 * mu1 * dn2 + mu2 * mu2 * reg["dn"])
    return pri / den, dual / dden


def run_fs(pb):
    """FS-MD in exact rational arithmetic (see the module header)."""
    one = Q(1)
    H, W_, J = pb["H"], pb["W"], pb["J"]
    n = H * W_
    zero = one * 0
    h = pb["kernel"]
    m = [one * v for v in pb["mask"]]
    y = list(pb["y"])
    lam, mu1, mu2 = pb["lam"], pb["mu1"], pb["mu2"]
    tau = lam / mu2
    A = conv_matrix(h, H, W_, one)
    P = [row for band in haar_bands(H, W_, J, one) for row in band]      # d x n analysis
    Wm = transpose(P)                                                   # n x d synthesis W = P^T
    AW = matmul(A, Wm)
    AWt = transpose(AW)
    d = len(P)
    N = [scale(mu1, row) for row in matmul(AWt, AW)]
    for i in range(d):
        N[i][i] += mu2
    fac = lu_factor(N)
    u1, d1 = [zero] * n, [zero] * n
    u2, d2 = [zero] * d, [zero] * d
    out, res, z = {}, {}, None
    for k in range(1, pb["iters"] + 1):
        u1_prev, u2_prev = u1, u2
        rhs = add(scale(mu1, matvec(AWt, add(u1, d1))), scale(mu2, add(u2, d2)))
        z = lu_solve(fac, rhs)
        AWz = matvec(AW, z)
        v1 = [a - b for a, b in zip(AWz, d1)]
        u1 = [(mi * yi + mu1 * vi) / (mi + mu1) for mi, yi, vi in zip(m, y, v1)]
        d1 = [b - (a - u) for b, a, u in zip(d1, AWz, u1)]
        v2 = [a - b for a, b in zip(z, d2)]
        u2 = [(abs(a) - tau) * (1 if a > 0 else -1) if abs(a) > tau else zero for a in v2]
        d2 = [b - (a - u) for b, a, u in zip(d2, z, u2)]
        if k in pb["record"]:
            out[k] = matvec(Wm, z)
            if k >= 2:
                res[k] = residuals(AWz, [z], u1, [u2], d1, [d2], u1_prev, [u2_prev], mu1, mu2)
    AWz = matvec(AW, z)
    fit = sum(((mi * (yi - a)) ** 2 for mi, yi, a in zip(m, y, AWz)), zero) / 2
    return out, fit + lam * sum((abs(a) for a in z), zero), res


def run(pb):
    if pb.get("method") == "fs":
        return run_fs(pb)
    reg = pb["reg"]
    one = Q(1) if reg == "fa" else Decimal(1)
    cv = (lambda q: q) if reg == "fa" else (lambda q: Decimal(q.numerator) / Decimal(q.denominator))
    H, W = pb["H"], pb["W"]
    n = H * W
    h = [[cv(v) for v in row] for row in pb["kernel"]]
    m = [one * v for v in pb["mask"]]
    y = [cv(v) for v in pb["y"]]
    lam, mu1, mu2 = cv(pb["lam"]), cv(pb["mu1"]), cv(pb["mu2"])
    tau = lam / mu2
    zero = one * 0

    A = conv_matrix(h, H, W, one)
    At = transpose(A)
    if reg == "tv":
        R = list(diff_matrices(H, W, one))
    else:
        R = haar_bands(H, W, pb["J"], one)
    Rt = [transpose(B) for B in R]
    # normal matrix of the z-step: mu1 A^T A + mu2 sum_b R_b^T R_b
    N = [scale(mu1, row) for row in matmul(At, A)]
    for B, Bt in zip(R, Rt):
        BtB = matmul(Bt, B)
        N = [add(row, scale(mu2, brow)) for row, brow in zip(N, BtB)]

    fac = lu_factor(N)
    cg = pb.get("method", "md") == "cg"
    if cg:
        # Reeves-Sorel variants: H1 = M A. C^{-1} = A^T A + gamma R^T R (dense),
        # B = the rows of A at the unobserved pixels, boundary system
        # S v = v - B C B^T v, one CG step per iteration from the previous v
        gamma = mu2 / mu1
        NC = matmul(At, A)
        for B_, Bt_ in zip(R, Rt):
            BtB = matmul(Bt_, B_)
            NC = [add(row, scale(gamma, brow)) for row, brow in zip(NC, BtB)]
        facC = lu_factor(NC)
        unobs = [i for i in range(n) if m[i] == 0]
        Brows = [A[i] for i in unobs]

        def Bt_of(v):   # B^T v as an n-vector
            out = [zero] * n
            for vj, row in zip(v, Brows):
                out = [o + vj * a for o, a in zip(out, row)]
            return out

        def S_of(v):
            w = lu_solve(facC, Bt_of(v))
            return [vj - sum((a * b for a, b in zip(row, w)), zero) for vj, row in zip(v, Brows)]

        vcg = [zero] * len(unobs)
    u1, d1 = [zero] * n, [zero] * n
    ur = [[zero] * n for _ in R]
    dr = [[zero] * n for _ in R]
    out = {}
    res = {}
    z = None
    for k in range(1, pb["iters"] + 1):
        u1_prev, ur_prev = u1, ur
        if not cg:
            rhs = scale(mu1, matvec(At, add(u1, d1)))
            for Bt, ub, db in zip(Rt, ur, dr):
                rhs = add(rhs, scale(mu2, matvec(Bt, add(ub, db))))
            z = lu_solve(fac, rhs)
            Az = matvec(A, z)
            v1 = [a - d for a, d in zip(Az, d1)]
            u1 = [(mi * yi + mu1 * vi) / (mi + mu1) for mi, yi, vi in zip(m, y, v1)]
            d1 = [d - (a - u) for d, a, u in zip(d1, Az, u1)]
        else:
            # r = mu1 A^T M^T zeta1 + mu2 R^T zeta_R (TV); A^T M^T zeta1 + gamma R^T zeta_R (FA)
            w1 = mu1 if reg == "tv" else one
            w2 = mu2 if reg == "tv" else gamma
            rhs = scale(w1, matvec(At, [mi * a for mi, a in zip(m, add(u1, d1))]))
            for Bt, ub, db in zip(Rt, ur, dr):
                rhs = add(rhs, scale(w2, matvec(Bt, add(ub, db))))
            t = lu_solve(facC, rhs)
            b = [sum((a * c for a, c in zip(row, t)), zero) for row in Brows]
            cres = [bi - si for bi, si in zip(b, S_of(vcg))]
            rr = sum((a * a for a in cres), zero)
            if rr != 0:
                q = S_of(cres)
                pq = sum((a * c for a, c in zip(cres, q)), zero)
                if pq > 0:
                    al = rr / pq
                    vcg = [vj + al * rj for vj, rj in zip(vcg, cres)]
            wz = add(t, lu_solve(facC, Bt_of(vcg)))
            z = [a / w1 for a in wz]
            Az = [mi * a for mi, a in zip(m, matvec(A, z))]      # M A z (zero off the mask)
            u1 = [mi * (yi + mu1 * (a - d)) / (1 + mu1) for mi, yi, a, d in zip(m, y, Az, d1)]
            d1 = [d - (a - u) for d, a, u in zip(d1, Az, u1)]
        Rz = [matvec(B, z) for B in R]
        vr = [[a - d for a, d in zip(Rb, db)] for Rb, db in zip(Rz, dr)]
        if reg == "tv":
            vh, vv = vr
            uh, uv = [], []
            for a, b in zip(vh, vv):
                rho2 = a * a + b * b
                rho = rho2.sqrt() if rho2 > 0 else zero
                if rho > tau:
                    f = (rho - tau) / rho
                    uh.append(a * f)
                    uv.append(b * f)
                else:
                    uh.append(zero)
                    uv.append(zero)
            ur = [uh, uv]
        else:
            ur = [[(abs(a) - tau) * (1 if a > 0 else -1) if abs(a) > tau else zero for a in vb] for vb in vr]
        dr = [[d - (a - u) for d, a, u in zip(db, Rb, ub)] for db, Rb, ub in zip(dr, Rz, ur)]
        if k in pb["record"]:
            out[k] = list(z)
            if k >= 2:
                res[k] = residuals(Az, Rz, u1, ur, d1, dr, u1_prev, ur_prev, mu1, mu2)
    # objective at the last z: 1/2 ||M (y - A z)||^2 + lambda * regulariser
    Az = matvec(A, z)
    fit = sum(((mi * (yi - a)) ** 2 for mi, yi, a in zip(m, y, Az)), zero) / 2
    Rz = [matvec(B, z) for B in R]
    if reg == "tv":
        pen = zero
        for a, b in zip(*Rz):
            s2 = a * a + b * b
            pen += s2.sqrt() if s2 > 0 else zero
    else:
        pen = sum((abs(a) for Rb in Rz for a in Rb), zero)
    return out, fit + lam * pen, res


def _dec(v):
    if isinstance(v, Q):
        v = Decimal(v.numerator) / Decimal(v.denominator)
    if v == 0:
        return "0"
    return format(v, ".25e")


def write(pb, zs, obj, res):
    path = os.path.join(HERE, pb["name"] + ".txt")
    if pb.get("method") == "fs":
        cite = ("FS-MD: Alg. 2 with H1 = A W, H2 = I (eqs. (13), (14)), the z-step of eq. (17), data step eq. (40), "
                "soft threshold eq. (16) on the coefficients, objective eq. (35), Sec. IV-C")
    elif pb.get("method", "md") == "cg":
        cite = ("TV-CG: Alg. 3 with A replaced by M A, the z-step of eq. (51) with one warm-started CG step, "
                "Sec. IV-D" if pb["reg"] == "tv" else
                "FA-CG: Alg. 2 with H1 = M A (eq. (45)), the z-step of eq. (47) with one warm-started CG step, "
                "Sec. IV-C")
    else:
        cite = ("TV-MD: Alg. 3 with the z-step of eq. (33) and the data step of eq. (49), Sec. IV-D"
                if pb["reg"] == "tv" else
                "FA-MD: Alg. 2 with the z-step of eqs. (24)-(25), data step eq. (40), soft threshold eq. (16), "
                "Sec. IV-C")
    arith = "60-digit decimal" if pb["reg"] == "tv" else "exact rational"
    lines = [
        f"# {cite}.",
        f"# Cold start, dense explicit operators, {arith} arithmetic; written by tests/golden/make_golden.py.",
        "# Values are row-major; inputs are exact fractions; z values carry 26 significant digits.",
        f"reg {pb['reg']}",
        f"method {pb.get('method', 'md')}",
        f"levels {pb.get('J', 0)}",
        f"shape {pb['H']} {pb['W']}",
        "kernel " + " ".join(str(v) for row in pb["kernel"] for v in row),
        "mask " + " ".join(str(v) for v in pb["mask"]),
        "y " + " ".join(str(v) for v in pb["y"]),
        f"lambda {pb['lam']}",
        f"mu1 {pb['mu1']}",
        f"mu2 {pb['mu2']}",
        f"iters {pb['iters']}",
    ]
    for k in sorted(zs):
        lines.append(f"z {k} " + " ".join(_dec(v) for v in zs[k]))
    for k in sorted(res):
        lines.append(f"residual {k} {_dec(res[k][0])} {_dec(res[k][1])}")
    lines.append(f"objective {pb['iters']} {_dec(obj)}")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    return path


def main():
    for make in PROBLEMS:
        pb = make()
        zs, obj, res = run(pb)
        print(write(pb, zs, obj, res))


if __name__ == "__main__":
    main()
