"""Krylov solvers and the block Gauss-Seidel iteration (oracle; test infrastructure only).

Sec. 4.2: B_T is nonsymmetric, so it is used with GMRes (Saad-Schultz);
B_D is SPD and used with CG.  Sec. 6: zero initial guess and a stop on the
relative residual in the Euclidean norm; GMRes restarted every r steps.

Readings taken here: right preconditioning (the analysis studies A B_T^{-1});
the flexible variant (FGMRES) keeps the preconditioned vectors z_j so that a
preconditioner which is not exactly linear (a reduced-precision V-cycle)
still yields x = x0 + Z y; the Arnoldi basis is built by modified
Gram-Schmidt, the small least-squares problem by Givens rotations, and the
stop test is the true residual ||F - A x|| / ||F|| recomputed whenever the
recurrence estimate falls below the tolerance or a cycle ends.

Sec. 4.2 also names GPCG (Blaheta) for the nonsymmetric B_T with the
symmetric A; GPCG[1] keeps one previous direction: the new direction is the
preconditioned residual A-orthogonalised against the last direction only,
p_{k+1} = z_{k+1} - ((A p_k, z_{k+1}) / (A p_k, p_k)) p_k, with
alpha_k = (r_k, p_k) / (A p_k, p_k).  For a symmetric preconditioner these
are the conjugate gradient iterates.  Sec. 6 (Table 3) also reports the block
Gauss-Seidel iteration x_{k+1} = x_k + B_T^{-1}(F - A x_k) (Sec. 4.2).
"""

import numpy as np


def fgmres(A, F, M, restart=30, tol=1e-8, max_it=1000, x0=None):
    """Right-preconditioned flexible GMRES(restart).

    A, M: callables on flat float64 vectors.  Returns (x, info).
    """
    F = np.asarray(F, dtype=np.float64).ravel()
    nF = np.linalg.norm(F)
    x = np.zeros_like(F) if x0 is None else np.asarray(x0, dtype=np.float64).ravel().copy()
    info = dict(iters=0, restarts=0, est=[], true=[], converged=False)
    if nF == 0.0:
        info["converged"] = True
        return x, info
    r = F - A(x)
    beta = np.linalg.norm(r)
    info["true"].append(beta / nF)
    if beta / nF < tol:
        info["converged"] = True
        return x, info
    while info["iters"] < max_it:
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        jlast = 0
        for j in range(restart):
            z = M(V[j])
            Z.append(z)
            w = A(z)
            for i in range(j + 1):
                H[i, j] = np.dot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            breakdown = H[j + 1, j] == 0.0
            if not breakdown:
                V.append(w / H[j + 1, j])
            # apply previous rotations, then form the new one
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            info["iters"] += 1
            info["est"].append(abs(g[j + 1]) / nF)
            jlast = j
            if abs(g[j + 1]) / nF < tol or breakdown or info["iters"] >= max_it:
                break
        k = jlast + 1
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        for i in range(k):
            x = x + y[i] * Z[i]
        r = F - A(x)
        beta = np.linalg.norm(r)
        info["true"].append(beta / nF)
        if beta / nF < tol:
            info["converged"] = True
            break
        info["restarts"] += 1
    return x, info


def gmres_left(A, F, M, restart=10, tol=1e-10, max_it=1000):
    """Left-preconditioned GMRES(restart) on M A x = M F from x = 0.

    The stop test is the relative residual of the preconditioned system,
    ||M (F - A x)|| / ||M F|| < tol: the running estimate from the Givens
    rotations inside a cycle, the recomputed value at the end of each cycle.
    (Reading of Sec. 6's GMRes(10): preconditioning from the left with the
    tolerance on the preconditioned residual, the convention of the MATLAB
    environment the section names.)  Returns (x, info), info["true"] holding
    ||F - A x|| / ||F|| after each cycle.
    """
    F = np.asarray(F, dtype=np.float64).ravel()
    x = np.zeros_like(F)
    MF = M(F)
    nMF = np.linalg.norm(MF)
    nF = np.linalg.norm(F)
    info = dict(iters=0, restarts=0, est=[], true=[], converged=False)
    if nMF == 0.0:
        info["converged"] = True
        return x, info
    while info["iters"] < max_it:
        r = M(F - A(x))
        beta = np.linalg.norm(r)
        if beta / nMF < tol:
            info["converged"] = True
            break
        V = [r / beta]
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        k = 0
        for j in range(restart):
            w = M(A(V[j]))
            for i in range(j + 1):
                H[i, j] = np.dot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0.0:
                V.append(w / H[j + 1, j])
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            info["iters"] += 1
            info["est"].append(abs(g[j + 1]) / nMF)
            k = j + 1
            if abs(g[j + 1]) / nMF < tol or len(V) == j + 1 or info["iters"] >= max_it:
                break
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        for i in range(k):
            x = x + y[i] * V[i]
        info["true"].append(np.linalg.norm(F - A(x)) / nF)
        if np.linalg.norm(M(F - A(x))) / nMF < tol:
            info["converged"] = True
            break
        info["restarts"] += 1
    return x, info


def pcg(A, F, M, tol=1e-8, max_it=1000, x0=None):
    """Preconditioned conjugate gradients with an SPD preconditioner M."""
    F = np.asarray(F, dtype=np.float64).ravel()
    nF = np.linalg.norm(F)
    x = np.zeros_like(F) if x0 is None else np.asarray(x0, dtype=np.float64).ravel().copy()
    info = dict(iters=0, est=[], true=[], converged=False)
    r = F - A(x)
    if np.linalg.norm(r) / nF < tol:
        info["converged"] = True
        return x, info
    z = M(r)
    pvec = z.copy()
    rz = np.dot(r, z)
    while info["iters"] < max_it:
        q = A(pvec)
        alpha = rz / np.dot(pvec, q)
        x = x + alpha * pvec
        r = r - alpha * q
        info["iters"] += 1
        rel = np.linalg.norm(r) / nF
        info["est"].append(rel)
        if rel < tol:
            rt = np.linalg.norm(F - A(x)) / nF
            info["true"].append(rt)
            if rt < tol:
                info["converged"] = True
                break
        z = M(r)
        rz_new = np.dot(r, z)
        pvec = z + (rz_new / rz) * pvec
        rz = rz_new
    return x, info


def gpcg1(A, F, M, tol=1e-8, max_it=1000, x0=None):
    """Generalised preconditioned CG with one stored direction (GPCG[1])."""
    F = np.asarray(F, dtype=np.float64).ravel()
    nF = np.linalg.norm(F)
    x = np.zeros_like(F) if x0 is None else np.asarray(x0, dtype=np.float64).ravel().copy()
    info = dict(iters=0, est=[], true=[], converged=False)
    r = F - A(x)
    if np.linalg.norm(r) / nF < tol:
        info["converged"] = True
        return x, info
    pvec = M(r)
    while info["iters"] < max_it:
        q = A(pvec)
        pq = np.dot(pvec, q)
        alpha = np.dot(r, pvec) / pq
        x = x + alpha * pvec
        r = r - alpha * q
        info["iters"] += 1
        rel = np.linalg.norm(r) / nF
        info["est"].append(rel)
        if rel < tol:
            rt = np.linalg.norm(F - A(x)) / nF
            info["true"].append(rt)
            if rt < tol:
                info["converged"] = True
                break
        z = M(r)
        pvec = z - (np.dot(q, z) / pq) * pvec
    return x, info


def block_gs(A, F, M, tol=1e-8, max_it=1000, x0=None):
    """Stationary iteration x <- x + M(F - A x) (block Gauss-Seidel when M = B_T^{-1})."""
    F = np.asarray(F, dtype=np.float64).ravel()
    nF = np.linalg.norm(F)
    x = np.zeros_like(F) if x0 is None else np.asarray(x0, dtype=np.float64).ravel().copy()
    info = dict(iters=0, est=[], true=[], converged=False)
    r = F - A(x)
    while info["iters"] < max_it:
        rel = np.linalg.norm(r) / nF
        info["true"].append(rel)
        if rel < tol:
            info["converged"] = True
            break
        x = x + M(r)
        r = F - A(x)
        info["iters"] += 1
    else:
        info["true"].append(np.linalg.norm(r) / nF)
        info["converged"] = info["true"][-1] < tol
    return x, info
