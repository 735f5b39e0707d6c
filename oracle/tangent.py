"""Frozen-path derivatives in mu and the kinetic scale lambda (oracle side; test infrastructure).

What is differentiated.  A walker's path is the sequence of shifted one-body matrices V_k
(fields and force-bias shifts, Sec. "Finite-Temperature AFQMC in the Grand Canonical
Ensemble") and weight exponents.  With that path held fixed, the slice propagators
B_k = K e^{V_k} K with K = exp(-dtau/2 (lambda eps + h - mu)) (eq. B), the constrained
products A_k = B_T^{n-k} B_k ... B_1 (eq. Abrenda), the overlap ratios
S_k = det(I + A_{k+1})^2 / det(I + A_k)^2, the phaseless weight
ln w = sum_k [Re ln S_k + Re(exponent_k) + ln cos theta_k] (eqs. import, phimport, theta)
and the local energy at tau = beta (Sec. "Uniform Electron Gas") are smooth functions of
(mu, lambda).  The trial B_T uses mu_T and does not depend on either.

How (all identities, no approximation):
  * Leibniz: the product of block upper-triangular [[B_k, dB_k], [0, B_k]] has dR_k in its
    off-diagonal block, so R and dR are carried together as one 2M x 2M product and
    stabilised by the same row-sorted QRCP stratification as the forward path.
  * The derivative of (I + A)^{-1} along dA is the off-diagonal block of the inverse of
    I + [[A, dA], [0, A]]; that inverse is taken by the same stable route (D_b/D_s split).
  * The overlap ratio of one slice is a well-conditioned M x M determinant,
    S_k^{1/2} = det(I + (B_{k+1} B_T^{-1} - I)(I - Gc_k)) with the cyclic Green's function
    Gc_k = (I + B_T R_k B_T^{n-k-1})^{-1}, so d ln S_k = 2 tr((I + Phi)^{-1} dPhi) with
    Phi = (B B_T^{-1} - I)(I - Gc), dPhi = dB B_T^{-1} (I - Gc) - (B B_T^{-1} - I) dGc.
  * Weighted means <O> = sum w O / sum w over live walkers:
    d<O> = sum w (dO + (O - <O>) d ln w) / sum w.
"""
import numpy as np

import scipy.linalg as sla

from . import path as _path
from .energy import local_energy


# --------------------------------------------------------------------------
# parameter directions
# --------------------------------------------------------------------------
def one_body_factors(sys, param):
    """K = exp(-dtau/2 (lambda eps + h - mu)) and dK/d(param), param in {"mu", "kscale"}."""
    kh = np.exp(-0.5 * sys.dtau * sys.h1_diag())
    if param == "mu":
        dkh = 0.5 * sys.dtau * kh
    elif param == "kscale":
        dkh = -0.5 * sys.dtau * sys.eps * kh
    else:
        raise ValueError("param must be 'mu' or 'kscale'")
    return kh, dkh


# --------------------------------------------------------------------------
# doubled (block upper-triangular) products
# --------------------------------------------------------------------------
def _inverse_of_graded(left, right_Q, right_D, right_T):
    """(I + diag(left) Q diag(D) T)^{-1} by row-sorted QRCP and the D_b/D_s split."""
    C = left[:, None] * right_Q * right_D[None, :]
    Q, D, T = _path.qdt_update(C, right_T, row_grading=left)
    G, _ = _path.greens_from_qdt(Q, D, T)
    return G


def literal_greens_doubled(sys, Qd, Dd, Td, k):
    """Inverse of I + diag(L, L) Rd with L = B_T^{n-k} and Rd = Qd diag(Dd) Td (2M x 2M)."""
    left = np.exp((sys.n_slices - k) * sys.log_trial_diag())
    return _inverse_of_graded(np.concatenate([left, left]), Qd, Dd, Td)


def cyclic_greens_doubled(sys, Qd, Dd, Td, k):
    """Inverse of I + diag(B_T, B_T) Rd diag(L, L) with L = B_T^{n-k-1}.

    Transposed, this is (I + diag(L,L) Td^T diag(Dd) (Qd^T diag(B_T,B_T)))^{-1}: the same
    left-graded form as the literal Green's function, with Td^T in the role of Q.
    """
    lt = sys.log_trial_diag()
    left = np.exp((sys.n_slices - k - 1) * lt)
    bt = np.exp(lt)
    L2, B2 = np.concatenate([left, left]), np.concatenate([bt, bt])
    return _inverse_of_graded(L2, Td.T, Dd, Qd.T * B2[None, :]).T


def path_tangent(sys, fwd, param):
    """Derivatives along one frozen path of a replayed walker.

    fwd: run_walker(..., record_path=True) output: the recorded path fwd["path"], the
    per-slice theta_k and the alive flags.  Returns dict(dlnS [n], dlogw, G and dG at
    tau = beta, dE1, dE2, dE, dN) in the spin-summed conventions of the local energy.
    """
    frozen = fwd["path"]
    M, n = sys.M, sys.n_slices
    kh, dkh = one_body_factors(sys, param)
    bt = np.exp(sys.log_trial_diag())
    Qd = np.eye(2 * M, dtype=np.complex128)
    Dd = np.ones(2 * M, dtype=np.complex128)
    Td = np.eye(2 * M, dtype=np.complex128)
    I = np.eye(M)
    dlnS = np.zeros(n, dtype=np.complex128)
    for k in range(n):
        E = sla.expm(frozen["V"][k])
        B = kh[:, None] * E * kh[None, :]
        dB = dkh[:, None] * E * kh[None, :] + kh[:, None] * E * dkh[None, :]
        # ratio of the step that inserts B_{k+1}, from the cyclic Green's function at R_k
        Gc = cyclic_greens_doubled(sys, Qd, Dd, Td, k)
        G0, dG0 = Gc[:M, :M], Gc[:M, M:]
        Wm = B / bt[None, :] - I
        Phi = Wm @ (I - G0)
        dPhi = (dB / bt[None, :]) @ (I - G0) - Wm @ dG0
        dlnS[k] = 2.0 * np.trace(np.linalg.solve(I + Phi, dPhi))
        # R_{k+1} = B_{k+1} R_k with its derivative, one stratification step
        Bd = np.block([[B, dB], [np.zeros_like(B), B]])
        Qd, Dd, Td = _path.qdt_update((Bd @ Qd) * Dd[None, :], Td)
    Gd = literal_greens_doubled(sys, Qd, Dd, Td, n)
    G, dG = Gd[:M, :M], Gd[:M, M:]
    dlogw = weight_tangent(fwd["theta"], fwd["alive"], dlnS)
    dkscale = 1.0 if param == "kscale" else 0.0
    e = energy_tangent(sys, G, dG, dkscale)
    return dict(dlnS=dlnS, dlogw=dlogw, G=G, dG=dG, **e)


def mu_tangent_closed_form(sys, fwd):
    """The mu direction in closed form.  K carries exp(dtau mu / 2) on both sides, so with the
    path frozen B_k(mu) = e^{dtau mu} B_k(0) and A_k = e^{k dtau mu} A_k(0):
      d ln det(I + A_k)/dmu = k dtau tr(I - G_k),  dG_n/dmu = -beta (I - G_n) G_n.
    fwd must hold the Green's function of every slice (keep_greens="all")."""
    Gs = fwd["greens_all"]
    n, dt = sys.n_slices, sys.dtau
    tr = np.array([np.trace(np.eye(sys.M) - G) for G in Gs])
    dell = dt * np.arange(n + 1) * tr
    dlnS = 2.0 * (dell[1:] - dell[:-1])
    G = Gs[-1]
    dG = -sys.beta * (np.eye(sys.M) - G) @ G
    dlogw = weight_tangent(fwd["theta"], fwd["alive"], dlnS)
    e = energy_tangent(sys, G, dG, 0.0)
    return dict(dlnS=dlnS, dlogw=dlogw, G=G, dG=dG, **e)


def weight_tangent(theta, alive, dlnS):
    """d ln w = sum over slices the walker survived of Re d ln S_k - tan(theta_k) Im d ln S_k
    (the exponent of eq. import is part of the frozen path; theta_k = Im ln S_k)."""
    d = 0.0
    for k in range(len(dlnS)):
        if not alive[k]:
            break
        d += dlnS[k].real - np.tan(theta[k]) * dlnS[k].imag
    return d


# --------------------------------------------------------------------------
# local energy and ensemble means
# --------------------------------------------------------------------------
def energy_tangent(sys, G, dG, dkscale):
    """Derivative of local_energy(sys, G) along G -> G + t dG and lambda -> lambda + t dkscale.

    With P = I - G^T and dP = -dG^T: E1 = 2 lambda sum eps P_KK, N = 2 sum P_KK,
    E2 = 1/2 sum_Q v_Q (4 r_Q r_-Q - 2 Lambda_Q) (Sec. "Uniform Electron Gas"), all at most
    quadratic in P, differentiated term by term.
    """
    M = sys.M
    P = np.eye(M) - G.T
    dP = -dG.T
    d, dd = np.diagonal(P), np.diagonal(dP)
    dE1 = 2.0 * dkscale * np.sum(sys.eps * d) + 2.0 * sys.kscale * np.sum(sys.eps * dd)
    dN = 2.0 * np.sum(dd)
    rho = np.array([P[sys.pairs[q]].sum() for q in range(sys.NQ)], dtype=np.complex128)
    drho = np.array([dP[sys.pairs[q]].sum() for q in range(sys.NQ)], dtype=np.complex128)
    dgamma = 4.0 * (drho * rho[sys.neg] + rho * drho[sys.neg])
    dlam = np.empty(sys.NQ, dtype=np.complex128)
    for q in range(sys.NQ):
        p, r = sys.pairs[q]
        dlam[q] = np.sum(dP[np.ix_(p, p)] * P[np.ix_(r, r)].T + P[np.ix_(p, p)] * dP[np.ix_(r, r)].T)
    dE2 = 0.5 * np.sum(sys.vq * (dgamma - 2.0 * dlam))
    return dict(dE1=dE1, dE2=dE2, dE=dE1 + dE2, dN=dN)


def ensemble_tangent(values, dvalues, logw, dlogw, status):
    """Weighted mean over live walkers and its derivative.

    values, dvalues: [W] complex; logw, dlogw: [W] real; status: [W] (0 = alive).
    Returns (<O>, d<O>) with <O> = sum w O / sum w.
    """
    live = (np.asarray(status) == _path.ALIVE) & np.isfinite(logw)
    lw = np.asarray(logw)[live]
    w = np.exp(lw - lw.max())
    O, dO, dl = np.asarray(values)[live], np.asarray(dvalues)[live], np.asarray(dlogw)[live]
    mean = np.sum(w * O) / np.sum(w)
    dmean = np.sum(w * (dO + (O - mean) * dl)) / np.sum(w)
    return mean, dmean


def walker_tangents(sys, z, params=("mu", "kscale")):
    """Forward path of one walker (recorded), then its frozen-path derivatives.

    Returns (fwd, {param: tangent dict}); fwd carries the final local energy in fwd["E"].
    """
    fwd = _path.run_walker(sys, z, record_path=True, energy_fn=local_energy)
    fwd["E"] = fwd["records"][-1]
    out = {p: path_tangent(sys, fwd, p) for p in params}
    return fwd, out


# --------------------------------------------------------------------------
# pathwise derivatives: the raw fields held fixed, the force bias recomputed
# --------------------------------------------------------------------------
def pathwise_tangent(sys, z, param):
    """Derivatives of one walker's path with the raw fields z held fixed while mu or lambda
    moves: besides the half-step factors K, the force bias of every slice follows G_k
    (Sec. "Phaseless approximation"), so the shifted one-body matrix V_k, its exponential and
    the exponent of eq. import all move.  This is what central differences of run_walker in
    (mu, lambda) measure.

    Per slice k, with the doubled product Rd = [[R, dR], [0, R]] (Leibniz) stratified as in the
    forward path:
      * G_k and dG_k are the blocks of the literal doubled inverse (I + diag(L, L) Rd)^{-1},
        L = B_T^{n-k}; dP = -dG^T gives dr_Q (per spin) and the shift derivatives
        dxbar_A = -sqrt(dtau) 2i a_Q (dr_Q + dr_-Q), dxbar_B = sqrt(dtau) 2 a_Q (dr_Q - dr_-Q);
      * dV is the one-body matrix of the coefficients of (-dxbar_A, -dxbar_B);
      * d e^V is the Frechet derivative, the off-diagonal block of expm([[V, dV], [0, V]]);
      * dB = dK e^V K + K e^V dK + K (d e^V) K;
      * d ln S_k from the cyclic Green's function as for the frozen path, and
        d(exponent_k) = sum [(x_A - xbar_A) dxbar_A + (x_B - xbar_B) dxbar_B].
    Returns (fwd, dict(dlnS, dexpo, dlogw, G, dG, dE1, dE2, dE, dN)).
    """
    fwd = _path.run_walker(sys, z, energy_fn=local_energy)
    fwd["E"] = fwd["records"][-1]
    M, n = sys.M, sys.n_slices
    kh, dkh = one_body_factors(sys, param)
    bt = np.exp(sys.log_trial_diag())
    sdt = np.sqrt(sys.dtau)
    Qd = np.eye(2 * M, dtype=np.complex128)
    Dd = np.ones(2 * M, dtype=np.complex128)
    Td = np.eye(2 * M, dtype=np.complex128)
    I = np.eye(M)
    dlnS = np.zeros(n, dtype=np.complex128)
    dexpo = np.zeros(n, dtype=np.complex128)
    Z = np.zeros((M, M), dtype=np.complex128)
    for k in range(n):
        Gd = literal_greens_doubled(sys, Qd, Dd, Td, k)
        G, dG = Gd[:M, :M], Gd[:M, M:]
        P, dP = np.eye(M) - G.T, -dG.T
        r = np.array([P[sys.pairs[q]].sum() for q in range(sys.NQ)], dtype=np.complex128)
        dr = np.array([dP[sys.pairs[q]].sum() for q in range(sys.NQ)], dtype=np.complex128)
        xbA, xbB = _path.force_bias(sys, P)
        dxbA = -sdt * 2.0 * 1j * sys.aq * (dr + dr[sys.neg])
        dxbB = sdt * 2.0 * sys.aq * (dr - dr[sys.neg])
        xA, xB = z[k].real, z[k].imag
        V = _path.one_body_matrix(sys, _path.hs_rho_coefficients(sys, xA - xbA, xB - xbB))
        dV = _path.one_body_matrix(sys, _path.hs_rho_coefficients(sys, -dxbA, -dxbB))
        dexpo[k] = np.sum((xA - xbA) * dxbA + (xB - xbB) * dxbB)
        big = sla.expm(np.block([[V, dV], [Z, V]]))
        E, dE = big[:M, :M], big[:M, M:]
        B = kh[:, None] * E * kh[None, :]
        dB = dkh[:, None] * E * kh[None, :] + kh[:, None] * E * dkh[None, :] + kh[:, None] * dE * kh[None, :]
        Gc = cyclic_greens_doubled(sys, Qd, Dd, Td, k)
        G0, dG0 = Gc[:M, :M], Gc[:M, M:]
        Wm = B / bt[None, :] - I
        Phi = Wm @ (I - G0)
        dPhi = (dB / bt[None, :]) @ (I - G0) - Wm @ dG0
        dlnS[k] = 2.0 * np.trace(np.linalg.solve(I + Phi, dPhi))
        Bd = np.block([[B, dB], [np.zeros_like(B), B]])
        Qd, Dd, Td = _path.qdt_update((Bd @ Qd) * Dd[None, :], Td)
    Gd = literal_greens_doubled(sys, Qd, Dd, Td, n)
    G, dG = Gd[:M, :M], Gd[:M, M:]
    d = 0.0
    for k in range(n):
        if not fwd["alive"][k]:
            break
        d += dlnS[k].real + dexpo[k].real - np.tan(fwd["theta"][k]) * dlnS[k].imag
    dkscale = 1.0 if param == "kscale" else 0.0
    e = energy_tangent(sys, G, dG, dkscale)
    return fwd, dict(dlnS=dlnS, dexpo=dexpo, dlogw=d, G=G, dG=dG, **e)


def kink_margin(fwd):
    """Smallest cos(theta_k) over the slices the walker survived: the weight is not
    differentiable where a slice's cos(theta) crosses 0 (the phaseless kill)."""
    c = [np.cos(fwd["theta"][k]) for k in range(len(fwd["theta"])) if fwd["alive"][k]]
    return min(c) if c else -1.0
