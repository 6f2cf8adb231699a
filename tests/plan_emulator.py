"""NumPy re-enactment of the kernels' arithmetic on a host-only plan's arrays.

Test helper only: it lets the CPU suite check the host factorisation (plan)
end to end against the oracle without a GPU.  It follows the same steps as
the device code -- interior generalized PCR per lane, interface RHS, block
PCR across lanes, back-substitution, and for P > 1 the workgroup-level
program -- but shares no code with it.
"""
import numpy as np


def _offsets(R, M, T, ilu=False):
    N = M - R
    k = 0
    dinv = (N * 2 * R) if ilu else (T * N * 2 * R)
    Lt = dinv + N
    Ut = Lt + R * R
    S = Ut + R * R
    Rm = S + N * R
    return dict(k=k, dinv=dinv, Lt=Lt, Ut=Ut, S=S, Rm=Rm, end=Rm + N * R)


def solve_segment(plan, b, seg=0):
    """b: (lines, S) -> x = D_seg^{-1} b by the lane scheme (cyclic or acyclic per plan)."""
    info = plan.info()
    R = info["r"]
    ilu = bool(plan.array(11, seg)[6])
    types = plan.array(3, seg).astype(int)
    starts = plan.array(4, seg).astype(int)
    L = len(types)
    flat = plan.array(0, seg)
    ntypes = int(types.max()) + 1
    M = None
    for cand in range(2 * R, 33):  # the block size fixes the register slots M
        Nc = cand - R
        Tc = 0
        while (1 << Tc) < Nc:
            Tc += 1
        if _offsets(R, cand, Tc, ilu)["end"] * ntypes == flat.size:
            M = cand
            break
    assert M is not None
    N = M - R
    T = 0
    while (1 << T) < N:
        T += 1
    o = _offsets(R, M, T, ilu)
    coef = flat.reshape(-1, o["end"])
    Tred = 0
    while (1 << Tred) < L:
        Tred += 1
    red = plan.array(1, seg).reshape(Tred, L, 2, R, R)
    wf = plan.array(2, seg).reshape(L, R, R)
    nl = b.shape[0]
    v = np.zeros((L, nl, M))
    m = np.diff(starts)
    for l in range(L):
        v[l, :, :m[l]] = b[:, starts[l]:starts[l + 1]]
    y = v[:, :, R:].copy()
    if ilu:  # banded elimination: forward with unit L, backward with U
        for l in range(L):
            lu = coef[types[l], o["k"]:o["dinv"]].reshape(N, 2 * R)
            dv = coef[types[l], o["dinv"]:o["Lt"]]
            for j in range(N):
                for q in range(1, R + 1):
                    if j - q >= 0:
                        y[l, :, j] -= lu[j, q - 1] * y[l, :, j - q]
            for j in range(N - 1, -1, -1):
                acc = y[l, :, j] * dv[j]
                for q in range(1, R + 1):
                    if j + q < N:
                        acc -= lu[j, R + q - 1] * y[l, :, j + q]
                y[l, :, j] = acc
        T = 0  # no PCR levels, no final scaling
    # interior generalized PCR
    for t in range(T):
        s = 1 << t
        yn = y.copy()
        for l in range(L):
            k = coef[types[l], o["k"]:o["dinv"]].reshape(T, N, 2 * R)
            for j in range(N):
                for q in range(1, R + 1):
                    if j - q * s >= 0:
                        yn[l, :, j] -= k[t, j, R - q] * y[l, :, j - q * s]
                    if j + q * s < N:
                        yn[l, :, j] -= k[t, j, R + q - 1] * y[l, :, j + q * s]
        y = yn
    for l in range(L if not ilu else 0):
        y[l] *= coef[types[l], o["dinv"]:o["Lt"]][None, :]
    # interface RHS
    xt = np.zeros((L, nl, R))
    for l in range(L):
        lp = (l - 1) % L
        nlp = m[lp] - R
        yprev = y[lp, :, nlp - R:nlp]
        Lt = coef[types[l], o["Lt"]:o["Ut"]].reshape(R, R)
        Ut = coef[types[l], o["Ut"]:o["S"]].reshape(R, R)
        xt[l] = v[l, :, :R] - yprev @ Lt.T - y[l, :, :R] @ Ut.T
    # block PCR across lanes
    for t in range(Tred):
        s = 1 << t
        xn = xt.copy()
        for l in range(L):
            xn[l] -= xt[(l + s) % L] @ red[t, l, 0].T + xt[(l - s) % L] @ red[t, l, 1].T
        xt = xn
    for l in range(L):
        xt[l] = xt[l] @ wf[l].T
    # back-substitution
    x = np.zeros_like(b)
    for l in range(L):
        S = coef[types[l], o["S"]:o["Rm"]].reshape(N, R)
        Rm = coef[types[l], o["Rm"]:o["end"]].reshape(N, R)
        xl = y[l] - xt[l] @ S.T - xt[(l + 1) % L] @ Rm.T
        x[:, starts[l]:starts[l] + R] = xt[l]
        x[:, starts[l] + R:starts[l + 1]] = xl[:, :m[l] - R]
    return x


def boundary_values(plan, b):
    """First and last R rows of y_i = D_i^{-1} b_i for every partition, as
    dot products of b_i's end windows with the plan's boundary rows."""
    info = plan.info()
    P, R, K = info["partitions"], info["r"], info["boundary_window"]
    ws = plan.array(7).astype(int)
    bf = plan.array(12).reshape(P, 2, R, K)
    yf, yl = [], []
    for i in range(P):
        seg = b[:, ws[i] + R:ws[i + 1]]
        N = seg.shape[1]
        # window rows 0..K-1 and N-K..N-1; rows outside the block (a block
        # shorter than the window) have zero weights
        first = np.zeros((b.shape[0], K))
        last = np.zeros((b.shape[0], K))
        first[:, :min(K, N)] = seg[:, :min(K, N)]
        last[:, max(0, K - N):] = seg[:, max(0, N - K):]
        yf.append(first @ bf[i, 0].T)
        yl.append(last @ bf[i, 1].T)
    return yf, yl


def solve(plan, b, seg=0):
    """x = A^{-1} b for (lines, n) b, following the plan's decomposition
    (seg = 1 selects the strided-launch lane layout of a one-partition plan)."""
    info = plan.info()
    P, R = info["partitions"], info["r"]
    if P == 1:
        return solve_segment(plan, b, seg)
    ws = plan.array(7).astype(int)
    SR = plan.array(5)
    LtUt = plan.array(6).reshape(P, 2, R, R)
    nl = b.shape[0]
    ys, sr = [], []
    off = 0
    for i in range(P):
        seg = b[:, ws[i] + R:ws[i + 1]]
        ys.append(solve_segment(plan, seg, i))
        Ni = ws[i + 1] - ws[i] - R
        sr.append((SR[off:off + Ni * R].reshape(Ni, R), SR[off + Ni * R:off + 2 * Ni * R].reshape(Ni, R)))
        off += 2 * Ni * R
    # phase A: the first and last R rows of y_i from the plan's boundary
    # rows of D_i^{-1} over their windows
    yf, yl = boundary_values(plan, b)
    xr = np.zeros((P, nl, R))
    for i in range(P):
        ip = (i - 1) % P
        xr[i] = b[:, ws[i]:ws[i] + R] - yl[ip] @ LtUt[i, 0].T - yf[i] @ LtUt[i, 1].T
    row_off = plan.array(8).astype(int)
    src = plan.array(9).astype(int)
    mats = plan.array(10).reshape(-1, R, R)
    nph = len(row_off) // (P + 1)
    for ph in range(nph):
        ro = row_off[ph * (P + 1):(ph + 1) * (P + 1)]
        xn = xr.copy()
        for j in range(P):
            if ro[j] == ro[j + 1]:
                continue
            acc = np.zeros((nl, R))
            for t in range(ro[j], ro[j + 1]):
                acc += xr[src[t]] @ mats[t].T
            xn[j] = acc
        xr = xn
    x = np.zeros_like(b)
    for i in range(P):
        Sg, Rg = sr[i]
        x[:, ws[i]:ws[i] + R] = xr[i]
        x[:, ws[i] + R:ws[i + 1]] = ys[i] - xr[i] @ Sg.T - xr[(i + 1) % P] @ Rg.T
    return x
