"""Oracle: the phi1 function and its action, computed from definitions.

TEST INFRASTRUCTURE ONLY (see the package docstring).

phi1(A) = sum_{i>=1} A^{i-1} / i! = A^{-1}(e^A - I)     (Sec. 3.2.2, after Eq. etd)

The action h*phi1(hM) v is read off the augmented exponential

    exp([[hM, h v], [0, 0]]) = [[e^{hM}, h phi1(hM) v], [0, 1]],

which follows term by term from the series above.  Two evaluations:

* tier A (dense): the exponential of the (N+1)^2 augmented matrix by Taylor
  scaling-and-squaring; cross-checked against scipy.linalg.expm in the tests.
* tier B (sparse): the action exp(Atilde) e_{N+1} by a truncated Taylor series
  applied over s substeps with ||hM||_1 / s <= 1; cross-checked against
  scipy.sparse.linalg.expm_multiply in the tests.

phi2 and the increment h phi1(hM) f + h^2 phi2(hM) g of the non-autonomous
step (Sec. 3.2.3, Eq. nEERMg) are read off an exponential augmented by two
rows and columns, again in a dense and a sparse tier.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


def phi1_scalar(z):
    """phi1(z) = (e^z - 1)/z, with phi1(0) = 1 (Sec. 3.2.2), evaluated with
    expm1 so that small |z| keeps full relative accuracy."""
    z = np.asarray(z, dtype=np.float64)
    out = np.ones_like(z)
    nz = z != 0.0
    out[nz] = np.expm1(z[nz]) / z[nz]
    return out


def expm_taylor(A, degree: int = 20):
    """Dense matrix exponential: scale A by 2^-s so that ||A/2^s||_1 <= 1/2,
    sum the Taylor series to ``degree`` by Horner's rule, square s times.
    Truncation error <= (1/2)^(degree+1)/(degree+1)! * e^(1/2) relative."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    nrm = np.abs(A).sum(axis=0).max() if n else 0.0
    s = 0
    if nrm > 0.5:
        s = int(math.ceil(math.log2(nrm / 0.5)))
    X = A / (2.0 ** s)
    I = np.eye(n)
    E = I.copy()
    for k in range(degree, 0, -1):
        E = I + (X @ E) / k
    for _ in range(s):
        E = E @ E
    return E


def phi1_matrix(M):
    """phi1(M) as the top-right block of exp([[M, I], [0, 0]])."""
    M = np.asarray(M, dtype=np.float64)
    n = M.shape[0]
    big = np.zeros((2 * n, 2 * n))
    big[:n, :n] = M
    big[:n, n:] = np.eye(n)
    return expm_taylor(big)[:n, n:]


def _pow2_scale(x: float) -> float:
    """Nearest power of two to x (> 0), so rescaling is exact."""
    if x <= 0.0 or not np.isfinite(x):
        return 1.0
    return 2.0 ** round(math.log2(x))


def hphi1_action_dense(M, v, h):
    """Tier A: return h * phi1(h M) v from the augmented exponential.

    The last column is divided by an exact power of two eta ~ ||h v||_inf to
    keep the augmented matrix balanced, and the block is multiplied back."""
    M = np.asarray(M, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    n = M.shape[0]
    eta = _pow2_scale(float(np.abs(h * v).max()) if n else 1.0)
    aug = np.zeros((n + 1, n + 1))
    aug[:n, :n] = h * M
    aug[:n, n] = h * v / eta
    E = expm_taylor(aug)
    return E[:n, n] * eta


def phi1_action_dense(M, v, h):
    """phi1(h M) v (tier A); h must be nonzero."""
    return hphi1_action_dense(M, v, h) / h


def hphi1_action_taylor(M, v, h, tol: float = 1e-18, max_terms: int = 200):
    """Tier B: h * phi1(h M) v for sparse M as the first N entries of
    exp(Atilde) e_{N+1}, Atilde = [[hM, hv], [0, 0]].

    exp(Atilde) = exp(Atilde/s)^s with s = ceil(||hM||_1); each factor is
    applied to the current vector y = [u; 1] by the Taylor series
    sum_k (Atilde/s)^k y / k!, truncated once two consecutive terms are below
    tol * ||y||_inf.  Atilde y = [hM u + h v * y_last; 0] and y_last stays 1.
    """
    M = sp.csr_matrix(M)
    v = np.asarray(v, dtype=np.float64)
    n = M.shape[0]
    hM = (h * M).tocsr()
    hv = h * v
    nrm = float(abs(hM).sum(axis=0).max()) if n else 0.0
    s = max(1, int(math.ceil(nrm)))
    u = np.zeros(n)
    for _ in range(s):
        # y = [u; 1]; term_0 = y
        term_u = u.copy()
        term_last = 1.0
        acc = u.copy()
        prev_small = False
        for k in range(1, max_terms + 1):
            new_u = (hM @ term_u + hv * term_last) / (s * k)
            term_u, term_last = new_u, 0.0
            acc += term_u
            small = np.abs(term_u).max() <= tol * np.abs(acc).max()
            if small and prev_small:
                break
            prev_small = small
        u = acc
    return u


# --------------------------------------------------------------------------
# phi2 and the non-autonomous action (Sec. 3.2.3, Eq. nEERMg)
# --------------------------------------------------------------------------

def phi2_scalar(z):
    """phi2(z) = (phi1(z) - phi1(0)) / z = (e^z - 1 - z) / z^2, phi2(0) = 1/2
    (Sec. 3.2.3, the recurrence of the phi functions).  Where |z| < 1 the
    series sum_{k>=0} z^k / (k+2)! is summed to 25 terms instead, which has
    no cancellation."""
    z = np.asarray(z, dtype=np.float64)
    out = np.empty_like(z)
    small = np.abs(z) < 1.0
    zs = z[small]
    acc = np.zeros_like(zs)
    term = np.full_like(zs, 0.5)
    for k in range(25):
        acc += term
        term = term * zs / (k + 3)
    out[small] = acc
    zl = z[~small]
    out[~small] = (np.expm1(zl) - zl) / (zl * zl)
    return out


def nonautonomous_action_dense(M, f, g, h):
    """Tier A: h phi1(h M) f + h^2 phi2(h M) g, the increment of Eq. nEERMg.

    It is the first N entries of the last column of exp(K) with

        K = [[h M, h^2 g, h f],
             [0,   0,     1  ],
             [0,   0,     0  ]]:

    y(s) = exp(s K) e_{N+2} has last entry 1 and middle entry s, and its top
    block solves u' = h M u + h f + s h^2 g from u(0) = 0, so
    u(1) = int_0^1 e^{(1-s) h M} (h f + s h^2 g) ds, which is the stated sum
    by the integral definition of phi_1 and phi_2.  The last two columns are
    divided by an exact power of two eta ~ max(|h f|, |h^2 g|) to keep K
    balanced, and the block is multiplied back."""
    M = np.asarray(M, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    n = M.shape[0]
    big = max(float(np.abs(h * f).max()), float(np.abs(h * h * g).max())) if n else 1.0
    eta = _pow2_scale(big)
    K = np.zeros((n + 2, n + 2))
    K[:n, :n] = h * M
    K[:n, n] = h * h * g / eta
    K[:n, n + 1] = h * f / eta
    K[n, n + 1] = 1.0
    E = expm_taylor(K)
    return E[:n, n + 1] * eta


def nonautonomous_action_taylor(M, f, g, h, tol: float = 1e-18, max_terms: int = 200):
    """Tier B: the same increment for sparse M as the top block of
    exp(K) e_{N+2} (K as in the dense tier), applied as exp(K/s)^s with
    s = ceil(||h M||_1) by the Taylor series of each factor on y = [u; a; b]:
    K y = [h M u + h^2 g a + h f b; b; 0].  A series stops once two
    consecutive terms of the u block are below tol * ||acc_u||_inf."""
    M = sp.csr_matrix(M)
    f = np.asarray(f, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    n = M.shape[0]
    hM = (h * M).tocsr()
    hf = h * f
    h2g = h * h * g
    nrm = float(abs(hM).sum(axis=0).max()) if n else 0.0
    s = max(1, int(math.ceil(nrm)))
    u = np.zeros(n)
    a, b = 0.0, 1.0
    for _ in range(s):
        tu, ta, tb = u.copy(), a, b
        acc_u, acc_a = u.copy(), a
        prev_small = False
        for k in range(1, max_terms + 1):
            nu = (hM @ tu + h2g * ta + hf * tb) / (s * k)
            na = tb / (s * k)
            tu, ta, tb = nu, na, 0.0
            acc_u += tu
            acc_a += ta
            small = np.abs(tu).max() <= tol * np.abs(acc_u).max()
            if small and prev_small and ta == 0.0:
                break
            prev_small = small
        u, a = acc_u, acc_a
    return u
