"""Block flexible GMRES, CPU side.

TEST INFRASTRUCTURE ONLY (oracle): only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it; it shares no code with the GPU
library.

The paper's experiments (section 4) solve s right-hand sides together by
block restarted FGMRES(m) (Calandra, Gratton, Langou, Pinel and Vasseur,
"Flexible variants of block restarted GMRES methods with application to
geophysics", 2012) with block size s = 10 and m = 10.  One cycle from X:
  R = B - A X = V_1 beta                 (thin QR, V_1 orthonormal N x s)
  for j = 1..m:
      Z_j = Prec(V_j)                    (column by column; Prec may vary)
      W = A Z_j
      H_ij = V_i^H W,  W -= V_i H_ij     (block modified Gram-Schmidt, i <= j)
      W = V_{j+1} H_{j+1,j}              (thin QR)
      Y_j = argmin || E_1 beta - Hbar_j Y ||_F   (Hbar_j: (j+1)s x js)
      the column norms of E_1 beta - Hbar_j Y_j are the residual norms
  X += [Z_1 .. Z_j] Y_j.
Each cycle restarts from the true residual; a right-hand side counts as
converged when its true relative residual ||b_k - A x_k|| / ||b_k|| <= tol,
and a cycle ends early when every column's estimate is below tol.  FP64
throughout; numpy's QR and least squares serve as the small dense steps.
"""
from __future__ import annotations

import numpy as np

from oracle import helm_oracle


def block_fgmres(hier, B, m=10, tol=1e-7, maxit=2000, prec=None):
    """B: complex [s, n, n].  prec: callable v -> z on one field, or None for
    the hierarchy's SL V-cycle.  Returns (X [s, n, n], dict with the number
    of block iterations, the cycles, the per-column true relative residuals
    and the per-column residual-estimate histories (relative to ||b_k||))."""
    kap, gam, om = hier.kappa0, hier.gamma0, hier.omega
    s, n = B.shape[0], B.shape[-1]
    N = n * n
    P = prec if prec is not None else hier.vcycle
    Bm = np.asarray(B, dtype=np.complex128).reshape(s, N).T           # N x s
    bn = np.linalg.norm(Bm, axis=0)
    X = np.zeros_like(Bm)
    A = lambda v: helm_oracle.apply(kap, gam, om, v.reshape(n, n)).ravel()
    its, cycles = 0, 0
    hist = [[1.0] for _ in range(s)]
    while True:
        R = Bm - np.stack([A(X[:, k]) for k in range(s)], axis=1)
        rel = np.linalg.norm(R, axis=0) / np.where(bn > 0, bn, 1.0)
        if np.all(rel <= tol) or its >= maxit:
            break
        V1, beta = np.linalg.qr(R)
        Vs, Zs = [V1], []
        Hbar = np.zeros(((m + 1) * s, m * s), dtype=np.complex128)
        E1b = np.zeros(((m + 1) * s, s), dtype=np.complex128)
        E1b[:s] = beta
        Y = None
        for j in range(m):
            Zj = np.stack([P(Vs[j][:, k].reshape(n, n)).ravel() for k in range(s)], axis=1)
            W = np.stack([A(Zj[:, k]) for k in range(s)], axis=1)
            for i in range(j + 1):
                Hij = Vs[i].conj().T @ W
                Hbar[i * s:(i + 1) * s, j * s:(j + 1) * s] = Hij
                W = W - Vs[i] @ Hij
            Vn, Hn = np.linalg.qr(W)
            Hbar[(j + 1) * s:(j + 2) * s, j * s:(j + 1) * s] = Hn
            Vs.append(Vn)
            Zs.append(Zj)
            its += 1
            k1 = (j + 2) * s
            H = Hbar[:k1, :(j + 1) * s]
            Y = np.linalg.lstsq(H, E1b[:k1], rcond=None)[0]
            est = np.linalg.norm(E1b[:k1] - H @ Y, axis=0) / np.where(bn > 0, bn, 1.0)
            for k in range(s):
                hist[k].append(float(est[k]))
            if np.all(est <= tol) or its >= maxit:
                break
        Zall = np.concatenate(Zs, axis=1)
        X = X + Zall @ Y
        cycles += 1
    return X.T.reshape(s, n, n), dict(iterations=its, cycles=cycles, true_relres=rel.tolist(), hist=hist)
