"""Independent checkers for the oracle: a dense formulation of (mn1)/(qp)
built from the problem statement, solved with scipy.  No code here is shared
with the oracle's sweep."""
import numpy as np


def pidx(i, j):
    return j * (j - 1) // 2 + i


def dense_problem(n, w, d):
    """A, b, c, Wdiag for v = (x, f) following (mn1) and (qp).

    Row order: metric rows 3 t + o (colex triplet t), then pair rows 2 p + c."""
    npairs = n * (n - 1) // 2
    rows, rhs = [], []
    # metric rows in colex triplet order (k, then j, then i), orientations 0..2
    colex = ((i, j, k) for k in range(n) for j in range(k) for i in range(j))
    for i, j, k in colex:
        pij, pik, pjk = pidx(i, j), pidx(i, k), pidx(j, k)
        for L, S1, S2 in ((pij, pik, pjk), (pik, pij, pjk), (pjk, pij, pik)):
            a = np.zeros(2 * npairs)
            a[L] += 1.0
            a[S1] -= 1.0
            a[S2] -= 1.0
            rows.append(a)
            rhs.append(0.0)
    for p in range(npairs):
        a = np.zeros(2 * npairs)
        a[p], a[npairs + p] = 1.0, -1.0
        rows.append(a)
        rhs.append(float(d[p]))
        a = np.zeros(2 * npairs)
        a[p], a[npairs + p] = -1.0, -1.0
        rows.append(a)
        rhs.append(-float(d[p]))
    A = np.array(rows).reshape(-1, 2 * npairs)
    b = np.array(rhs)
    c = np.concatenate([np.zeros(npairs), w])
    W = np.concatenate([w, w])
    return A, b, c, W


def qp_bruteforce(n, w, d, gamma):
    """Solve min c'v + 1/(2 gamma) v'Wv s.t. Av <= b: SLSQP, then an exact
    KKT solve on the detected active set.  Returns v."""
    from scipy.optimize import minimize
    A, b, c, W = dense_problem(n, w, d)
    H = W / gamma
    fun = lambda v: c @ v + 0.5 * v @ (H * v)
    jac = lambda v: c + H * v
    v0 = np.concatenate([np.asarray(d, float), np.zeros(len(w))])
    res = minimize(fun, v0, jac=jac, method="SLSQP",
                   constraints=[dict(type="ineq", fun=lambda v: b - A @ v, jac=lambda v: -A)],
                   options=dict(ftol=1e-15, maxiter=2000))
    v = res.x
    # primal active-set refinement: exact KKT solves on a working set, adding
    # the most violated row or dropping the most negative multiplier
    act = (b - A @ v) < 1e-7
    nv = len(v)
    for _ in range(200):
        Aa, ba = A[act], b[act]
        m = Aa.shape[0]
        K = np.zeros((nv + m, nv + m))
        K[:nv, :nv] = np.diag(H)
        K[:nv, nv:] = Aa.T
        K[nv:, :nv] = Aa
        sol = np.linalg.lstsq(K, np.concatenate([-c, ba]), rcond=None)[0]
        vk, lam = sol[:nv], sol[nv:]
        viol = A @ vk - b
        lmin = lam.min() if m else 0.0
        if lmin >= -1e-12 and viol.max() <= 1e-12:
            return vk
        idx = np.flatnonzero(act)
        if lmin < -1e-12:
            act[idx[np.argmin(lam)]] = False
        else:
            act[np.argmax(viol)] = True
    raise RuntimeError("active-set refinement did not settle")


def lp_optimum(n, w, d):
    """LP optimum of (mn1) via HiGHS."""
    from scipy.optimize import linprog
    A, b, c, _ = dense_problem(n, w, d)
    r = linprog(c, A_ub=A, b_ub=b, bounds=[(None, None)] * len(c), method="highs")
    assert r.status == 0
    return r.fun


def halfspace_projection(v, a, beta, Wdiag):
    """W-norm projection of v onto {u : a'u <= beta} (closed form)."""
    viol = a @ v - beta
    if viol <= 0:
        return v.copy()
    Winv_a = a / Wdiag
    return v - viol * Winv_a / (a @ Winv_a)


def dense_metric_rows(n):
    """The metric rows over x alone, in colex triplet order 3 t + o."""
    npairs = n * (n - 1) // 2
    rows = []
    for k in range(n):
        for j in range(k):
            for i in range(j):
                pij, pik, pjk = pidx(i, j), pidx(i, k), pidx(j, k)
                for L, S1, S2 in ((pij, pik, pjk), (pik, pij, pjk), (pjk, pij, pik)):
                    a = np.zeros(npairs)
                    a[L] += 1.0
                    a[S1] -= 1.0
                    a[S2] -= 1.0
                    rows.append(a)
    return np.array(rows).reshape(-1, npairs)


def nearness_bruteforce(n, w, dv):
    """min (1/2) sum w (x - d)^2 s.t. every metric row <= 0, by SLSQP and an
    exact KKT solve on the detected active set.  Returns x."""
    from scipy.optimize import minimize
    A = dense_metric_rows(n)
    w = np.asarray(w, float)
    dv = np.asarray(dv, float)
    fun = lambda x: 0.5 * np.sum(w * (x - dv) ** 2)
    jac = lambda x: w * (x - dv)
    res = minimize(fun, dv.copy(), jac=jac, method="SLSQP",
                   constraints=[dict(type="ineq", fun=lambda x: -A @ x, jac=lambda x: -A)],
                   options=dict(ftol=1e-15, maxiter=2000))
    x = res.x
    act = (-A @ x) < 1e-7
    nv = len(x)
    for _ in range(200):
        Aa = A[act]
        m = Aa.shape[0]
        K = np.zeros((nv + m, nv + m))
        K[:nv, :nv] = np.diag(w)
        K[:nv, nv:] = Aa.T
        K[nv:, :nv] = Aa
        sol = np.linalg.lstsq(K, np.concatenate([w * dv, np.zeros(m)]), rcond=None)[0]
        xk, lam = sol[:nv], sol[nv:]
        viol = A @ xk
        lmin = lam.min() if m else 0.0
        if lmin >= -1e-12 and viol.max() <= 1e-12:
            return xk
        idx = np.flatnonzero(act)
        if lmin < -1e-12:
            act[idx[np.argmin(lam)]] = False
        else:
            act[np.argmax(viol)] = True
    raise RuntimeError("active-set refinement did not settle")
