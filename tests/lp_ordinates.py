"""Deterministic solution of the Levermore-Pomraning (LP) equations that CLS
solves (Section 1 closure; Section 4: Algorithm A solves LP), for the
benchmark box of Section 2 reduced to the x axis.

TEST INFRASTRUCTURE: a noise-free second reference for the CLS oracle in
scattering cases. It shares no code with the oracle or the GPU library.

With psi_i = p_i <phi_i> the LP system is, per direction omega (Section 1,
closure p_ij = p_i / Lambda_i(omega)),
    omega . grad psi_i + (Sigma_i + r_i) psi_i
        = r_j psi_j + (c_i Sigma_i / W) int psi_i domega' + p_i S,
with r_i(omega) = 1 / Lambda_i(omega) the interface rate per unit path:
|mu| / Lambda_i in the slab (Sec. 4.1), sqrt(omega_x^2 + omega_y^2) / Lambda_i in
the extruded geometry (Sec. 4.2), 1 / Lambda_i in 3D (Sec. 4.3) and on the rod;
W = 4 pi (2 on the rod, directions +-x). Reflecting lateral faces and sources
uniform across them make the solution depend on x and the direction only.
Suite I: incident angular flux p_i / pi on x = 0 (unit incident current,
cosine law), suite II: uniform isotropic source of unit total strength.

Discretization: discrete ordinates (Gauss-Legendre in mu on each half range,
in the azimuth for the extruded geometry), x cells of width h, and per
direction and cell the exact solution of mu dpsi/dx = -A psi + q for a
constant source q (2x2 matrix exponential: a characteristic scheme, exactly
conservative). The scalar fluxes solve phi = K phi + b (K: one sweep of the
scattering source) by GMRES.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.linalg import expm
from scipy.sparse.linalg import LinearOperator, gmres


@dataclass
class LPResult:
    T: float
    R: float
    A: float              # absorption rate (balance: T + R + A = 1)
    total_flux: float     # integral of the scalar flux over x
    flux: np.ndarray      # bin-averaged scalar flux
    iterations: int


def _directions(geom: str, nmu: int, nphi: int):
    """Ordinates: mu (x-cosine), weight (sum W), chord factor g (rate = g / Lambda)."""
    if geom == "rod":
        return np.array([1.0, -1.0]), np.array([1.0, 1.0]), np.array([1.0, 1.0]), 2.0
    x, w = np.polynomial.legendre.leggauss(nmu)
    mu_half = 0.5 * (x + 1.0)
    w_half = 0.5 * w
    mus = np.concatenate([mu_half, -mu_half])
    if geom in ("slab", "cube3d"):
        ws = np.concatenate([w_half, w_half]) * 2.0 * np.pi
        g = np.abs(mus) if geom == "slab" else np.ones_like(mus)
        return mus, ws, g, 4.0 * np.pi
    if geom == "ext2d":
        # the sources are uniform in the azimuth phi about x and the chord factor
        # depends on cos^2 phi only, so one quarter [0, pi/2] (weight x 4) holds
        # the whole azimuthal integral; the factor's kink at cos phi = 0 (mu -> 0)
        # is then an end point, where Gauss-Legendre converges fast
        xp, wp = np.polynomial.legendre.leggauss(nphi)
        phi = 0.25 * np.pi * (xp + 1.0)   # [0, pi/2]
        wphi = 4.0 * 0.25 * np.pi * wp
        M, P = np.meshgrid(mus, phi, indexing="ij")
        WM, WP = np.meshgrid(np.concatenate([w_half, w_half]), wphi, indexing="ij")
        mu = M.ravel()
        # omega = (mu, sqrt(1-mu^2) cos phi, sqrt(1-mu^2) sin phi); z is the
        # extrusion axis: g = sqrt(omega_x^2 + omega_y^2)
        g = np.sqrt(mu * mu + (1.0 - mu * mu) * np.cos(P.ravel()) ** 2)
        return mu, (WM * WP).ravel(), g, 4.0 * np.pi
    raise ValueError(geom)


def solve(geom: str, sigma, c, lam, L: float, nbins: int, source: str = "face", nx: int = 2000,
          nmu: int = 64, nphi: int = 32, tol: float = 1e-11) -> LPResult:
    """LP solution for geometry 'rod', 'slab', 'ext2d' or 'cube3d' and source
    'face' or 0 (suite I), 'volume' or 1 (suite II)."""
    assert nx % nbins == 0
    source = {0: "face", 1: "volume"}.get(source, source)
    sig = np.asarray(sigma, float)
    cc = np.asarray(c, float)
    lm = np.asarray(lam, float)
    p = lm / lm.sum()
    mu, w, g, W = _directions(geom, nmu, nphi)
    h = L / nx
    D = len(mu)
    # per-direction 2x2 operators: A, E = expm(-A h/|mu|), Ainv, B = (|mu|/h) Ainv (I - E)
    A = np.zeros((D, 2, 2))
    A[:, 0, 0] = sig[0] + g / lm[0]
    A[:, 0, 1] = -g / lm[1]
    A[:, 1, 0] = -g / lm[0]
    A[:, 1, 1] = sig[1] + g / lm[1]
    E = np.array([expm(-A[d] * h / abs(mu[d])) for d in range(D)])
    Ainv = np.linalg.inv(A)
    I2 = np.eye(2)
    B = (np.abs(mu) / h)[:, None, None] * np.einsum("dij,djk->dik", Ainv, I2[None] - E)
    ImE = I2[None] - E
    fwd = mu > 0
    scat = cc * sig / W                   # per material: scattering source per unit phi_i

    if source == "face":
        psi_in = np.zeros((D, 2))
        psi_in[fwd] = p[None, :] * ((1.0 / np.pi) if geom != "rod" else 1.0)
        ext = np.zeros(2)
    elif source == "volume":
        psi_in = np.zeros((D, 2))
        ext = p / (L * W)
    else:
        raise ValueError(source)

    def sweep(phi_cells, with_external):
        """One transport sweep: cell scalar fluxes (nx, 2) from a source built on
        phi_cells (scattering) plus, optionally, the external source and the
        incident flux; also returns the exit currents."""
        q = scat[None, :] * phi_cells + (ext[None, :] if with_external else 0.0)     # (nx, 2)
        out = np.zeros((nx, 2))
        exits = {}
        for key, sel, order in (("T", fwd, range(nx)), ("R", ~fwd, range(nx - 1, -1, -1))):
            Ed, Bd, Ai, Im, wd = E[sel], B[sel], Ainv[sel], ImE[sel], w[sel]
            psi = psi_in[sel].copy() if with_external else np.zeros((int(sel.sum()), 2))
            for k in order:
                s = np.einsum("dij,j->di", Ai, q[k])
                avg = s + np.einsum("dij,dj->di", Bd, psi - s)
                out[k] += wd @ avg
                psi = np.einsum("dij,dj->di", Ed, psi) + np.einsum("dij,dj->di", Im, s)
            exits[key] = (np.abs(mu[sel]) * wd) @ psi.sum(axis=1)
        return out, exits

    b, _ = sweep(np.zeros((nx, 2)), True)
    n = 2 * nx

    def matvec(v):
        phi = v.reshape(nx, 2)
        k, _ = sweep(phi, False)
        return (phi - k).ravel()

    it = [0]

    def cb(_):
        it[0] += 1

    op = LinearOperator((n, n), matvec=matvec, dtype=float)
    sol, info = gmres(op, b.ravel(), rtol=tol, atol=0.0, restart=200, maxiter=2000, callback=cb,
                      callback_type="pr_norm")
    if info != 0:
        raise RuntimeError(f"GMRES did not converge ({info})")
    phi = sol.reshape(nx, 2)
    _, exits = sweep(phi, True)
    # the forward ordinates leave at x = L (T), the backward ones at x = 0 (R)
    T = float(exits["T"])
    R = float(exits["R"])
    absorb = float(h * np.sum(((1.0 - cc) * sig)[None, :] * phi))
    total = phi.sum(axis=1)
    flux = total.reshape(nbins, nx // nbins).mean(axis=1)
    return LPResult(T=T, R=R, A=absorb, total_flux=float(h * total.sum()), flux=flux, iterations=it[0])
