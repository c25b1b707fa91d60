"""Closed-form and deterministic solutions that pin the CLS oracle (test-only).

Nothing here is Monte Carlo and nothing here calls the oracle or the GPU library:
these are the exact expectations that CLS estimates in the special cases where
they have a plain definition.

* Levermore-Pomraning (LP) model, Section 1 of Larmier et al. (arXiv 1708.00765):
  the material-averaged transport equation with the closure p_ij = p_i / Lambda_i
  (Eq. for the LP closure). Section 4 states that CLS (Algorithm A) solves it
  formally, and that CLS is exact for pure absorbers.
* The rod (directions +-x) turns the LP model into a 4x4 linear ODE system in x;
  pure absorbers in slab, 2D extruded and 3D geometries reduce it to a 2x2 system
  along each straight path, integrated over the incidence law of suite I (Sec. 4).
* Homogeneous media (Sigma_0 = Sigma_1, c_0 = c_1) give the textbook two-stream rod
  formula and the exponential-integral formulas of the slab with an isotropic
  incident flux.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm
from scipy.sparse import lil_matrix
from scipy.sparse.linalg import spsolve
from scipy.special import expn


# ---------------------------------------------------------------------------
# homogeneous media
# ---------------------------------------------------------------------------
def rod_two_stream(sigma: float, c: float, L: float) -> tuple[float, float]:
    """Transmission and reflection of a homogeneous rod with unit incident current.

    psi+' = -a psi+ + b psi-,  psi-' = a psi- - b psi+  with a = Sigma (1 - c/2),
    b = c Sigma / 2, psi+(0) = 1, psi-(L) = 0; k = Sigma sqrt(1 - c).
    """
    a = sigma * (1.0 - c / 2.0)
    b = c * sigma / 2.0
    k = sigma * np.sqrt(max(1.0 - c, 0.0))
    if k * L < 1e-8:
        return 1.0 / (1.0 + a * L), a * L / (1.0 + a * L)
    D = k * np.cosh(k * L) + a * np.sinh(k * L)
    return k / D, b * np.sinh(k * L) / D


def slab_absorber_cosine(sigma: float, L: float, nbins: int):
    """Homogeneous pure absorber, isotropic incident flux (cosine-weighted current).

    T = 2 E3(Sigma L). The scalar flux per incident particle at depth x is
    phi(x) = 2 E2(Sigma x); its bin average over [x_k, x_k+1] is
    (2/Sigma)(E3(Sigma x_k) - E3(Sigma x_k+1)) / dx.
    """
    T = 2.0 * expn(3, sigma * L)
    edges = np.linspace(0.0, L, nbins + 1)
    dx = L / nbins
    e3 = expn(3, sigma * edges)
    flux = (2.0 / sigma) * (e3[:-1] - e3[1:]) / dx
    return T, flux


# ---------------------------------------------------------------------------
# rod: full LP model with scattering (4x4 system)
# ---------------------------------------------------------------------------
def _rod_lp_matrix(sigma, c, lam):
    """dF/dx = M F for F = (f0+, f1+, f0-, f1-), f_i^pm = p_i psi_i^pm.

    + direction:  f_i+' = -Sigma_i f_i+ - f_i+/Lambda_i + f_j+/Lambda_j + (c_i Sigma_i/2)(f_i+ + f_i-)
    - direction: -f_i-' = -Sigma_i f_i- - f_i-/Lambda_i + f_j-/Lambda_j + (c_i Sigma_i/2)(f_i+ + f_i-)
    """
    s = np.asarray(sigma, float)
    cc = np.asarray(c, float)
    lm = np.asarray(lam, float)
    P = np.array([[-1.0 / lm[0], 1.0 / lm[1]],
                  [1.0 / lm[0], -1.0 / lm[1]]])
    Cs = np.diag(cc * s / 2.0)
    B = -np.diag(s) + P + Cs
    M = np.zeros((4, 4))
    M[:2, :2] = B
    M[:2, 2:] = Cs
    M[2:, 2:] = -B
    M[2:, :2] = -Cs
    return M


def rod_lp(sigma, c, lam, L: float, nbins: int, substeps: int | None = None):
    """Exact LP solution on the rod with a unit current entering x=0 along +x.

    Returns (T, R, flux[nbins]) with flux the bin-averaged scalar flux
    f0+ + f1+ + f0- + f1- per incident particle. The two-point boundary value
    problem (f+(0) = p, f-(L) = 0) is solved stably by multiple shooting: the
    propagator expm(M h) on each of nbins*substeps sub-intervals (h small enough
    that |M| h stays below 4) links the nodal values in one sparse
    block-bidiagonal linear system; bin integrals of F use the Van Loan block
    exponential expm([[M, I], [0, 0]] h).
    """
    lm = np.asarray(lam, float)
    p = lm / lm.sum()
    M = _rod_lp_matrix(sigma, c, lam)
    if substeps is None:
        rho = np.abs(M).sum(axis=1).max()
        substeps = max(4, int(np.ceil(rho * L / nbins / 4.0)))
    n = nbins * substeps
    h = L / n
    E = expm(M * h)
    V = np.zeros((8, 8))
    V[:4, :4] = M
    V[:4, 4:] = np.eye(4)
    G = expm(V * h)[:4, 4:]            # integral_0^h expm(M t) dt
    N = 4 * (n + 1)
    A = lil_matrix((N, N))
    rhs = np.zeros(N)
    row = 0
    A[row, 0] = 1.0; rhs[row] = p[0]; row += 1          # f0+(0) = p0
    A[row, 1] = 1.0; rhs[row] = p[1]; row += 1          # f1+(0) = p1
    for k in range(n):
        for i in range(4):
            for j in range(4):
                A[row + i, 4 * k + j] = -E[i, j]
            A[row + i, 4 * (k + 1) + i] = 1.0
        row += 4
    A[row, 4 * n + 2] = 1.0; row += 1                   # f0-(L) = 0
    A[row, 4 * n + 3] = 1.0; row += 1                   # f1-(L) = 0
    F = spsolve(A.tocsc(), rhs).reshape(n + 1, 4)
    T = F[n, 0] + F[n, 1]
    R = F[0, 2] + F[0, 3]
    one = np.ones(4)
    sub = (F[:n] @ G.T) @ one
    flux = sub.reshape(nbins, substeps).sum(axis=1) / (L / nbins)
    return T, R, flux


# ---------------------------------------------------------------------------
# pure absorbers (c0 = c1 = 0): 2x2 system along each path
# ---------------------------------------------------------------------------
def _absorber_A(sigma, lam, q):
    """Per-unit-path attenuation/transfer matrix: chord rate q / Lambda_i."""
    s = np.asarray(sigma, float)
    lm = np.asarray(lam, float)
    return np.array([[s[0] + q / lm[0], -q / lm[1]],
                     [-q / lm[0], s[1] + q / lm[1]]])


def _gauss01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def markov_absorber(geom: str, sigma, lam, L: float, nbins: int, nmu: int = 400, nphi: int = 128):
    """Exact LP (= exact CLS) pure-absorber T and bin flux for the suite-I source.

    geom: 'rod' (direction +x, chord factor 1), 'slab' (x-cosine mu with density
    2 mu, chord factor |mu|), 'cube3d' (x-cosine density 2 mu, chord factor 1),
    'ext2d' (x-cosine mu' density 2 mu', azimuth phi' uniform about x, chord
    factor Q = sqrt(mu'^2 + (1-mu'^2) cos^2 phi')). Along a direction with
    x-cosine mu the survival vector after reaching depth x is
    expm(-A x / mu) p, A = [[S0 + q/L0, -q/L1], [-q/L0, S1 + q/L1]].
    The track length per unit depth is 1/mu, so the bin-averaged flux is
    (1/dx) 1^T A^-1 (expm(-A x_k/mu) - expm(-A x_k+1/mu)) p per direction.
    """
    lm = np.asarray(lam, float)
    p = lm / lm.sum()
    edges = np.linspace(0.0, L, nbins + 1)
    dx = L / nbins

    def per_direction(mu, q):
        A = _absorber_A(sigma, lam, q)
        Ainv = np.linalg.inv(A)
        Ek = [expm(-A * e / mu) @ p for e in edges]
        t = Ek[-1].sum()
        fl = np.array([(Ainv @ (Ek[k] - Ek[k + 1])).sum() for k in range(nbins)]) / dx
        return t, fl

    if geom == "rod":
        return per_direction(1.0, 1.0)
    mus, wmu = _gauss01(nmu)
    T = 0.0
    flux = np.zeros(nbins)
    if geom in ("slab", "cube3d"):
        for mu, w in zip(mus, wmu):
            q = mu if geom == "slab" else 1.0
            t, fl = per_direction(mu, q)
            T += w * 2.0 * mu * t
            flux += w * 2.0 * mu * fl
        return T, flux
    if geom == "ext2d":
        phis, wphi = _gauss01(nphi)
        for mu, w in zip(mus, wmu):
            for ph, wp in zip(phis, wphi):
                q = np.sqrt(mu * mu + (1.0 - mu * mu) * np.cos(2.0 * np.pi * ph) ** 2)
                t, fl = per_direction(mu, q)
                T += w * wp * 2.0 * mu * t
                flux += w * wp * 2.0 * mu * fl
        return T, flux
    raise ValueError(geom)


def atomic_mix(sigma, c, lam):
    """Atomic-mix homogenization (Section 2): Sigma_bar = sum p_i Sigma_i and
    c_bar Sigma_bar = sum p_i c_i Sigma_i."""
    lm = np.asarray(lam, float)
    p = lm / lm.sum()
    s = np.asarray(sigma, float)
    cc = np.asarray(c, float)
    sbar = float((p * s).sum())
    cbar = float((p * cc * s).sum()) / sbar
    return sbar, cbar
