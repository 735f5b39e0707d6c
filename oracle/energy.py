"""Local energy of one walker (oracle side; test infrastructure).

Sec. "Uniform Electron Gas": epsilon = E_M + E_1 + E_2 with
  E_1 = sum_K |K|^2/2 P_KK (times the kinetic scale lambda of H_1 = lambda T),
  E_2 = 1/(2 Omega) sum_{Q != 0} 4 pi / |Q|^2 (Gamma_Q - Lambda_Q),
  Gamma_Q = (sum_K1 P_{K1+Q,K1}) (sum_K2 P_{K2-Q,K2})        (Hartree),
  Lambda_Q = sum_{K1,K2} P_{K1+Q,K2} P_{K2-Q,K1}           (exchange),
evaluated with generalised Wick's theorem from P = I - G^T.  The printed
Gamma_Q has garbled second indices; Wick's theorem on the normal-ordered V_ee
fixes them as above.  Sums over spin: P is the per-spin block (both spins
equal), so E_1 and N carry 2, the Hartree term 4 (both spin pairs) and the
exchange term 2 (same spin only).
"""
import numpy as np


def local_energy(sys, G):
    """Return dict(E1, E2, E, N) (complex) for the per-spin Green's function G."""
    M = sys.M
    P = np.eye(M) - G.T
    d = np.diagonal(P)
    E1 = 2.0 * sys.kscale * np.sum(sys.eps * d)
    N = 2.0 * np.sum(d)
    rho = np.array([P[sys.pairs[q]].sum() for q in range(sys.NQ)], dtype=np.complex128)
    gamma = 4.0 * rho * rho[sys.neg]
    lam = np.empty(sys.NQ, dtype=np.complex128)
    for q in range(sys.NQ):
        p, r = sys.pairs[q]          # K_p - K_r = Q for every listed pair
        # Lambda_Q = sum_{i,j} P[p_i, p_j] P[r_j, r_i]  (K1 = r_i, K2 = p_j)
        lam[q] = np.sum(P[np.ix_(p, p)] * P[np.ix_(r, r)].T)
    E2 = 0.5 * np.sum(sys.vq * (gamma - 2.0 * lam))
    return dict(E1=E1, E2=E2, E=E1 + E2 + sys.E_M, N=N)


def local_energy_loops(sys, G):
    """The same estimator with explicit loops over K1, K2 (small bases only)."""
    M = sys.M
    P = np.eye(M) - G.T
    where = {tuple(v): i for i, v in enumerate(sys.nvec)}
    E1 = 2.0 * sys.kscale * sum(sys.eps[i] * P[i, i] for i in range(M))
    E2 = 0.0
    for q in range(sys.NQ):
        Q = tuple(sys.qvec[q])
        g1 = g2 = 0.0
        lam = 0.0
        for k1 in range(M):
            a = where.get(tuple(sys.nvec[k1] + Q))
            if a is not None:
                g1 += P[a, k1]
            for k2 in range(M):
                b = where.get(tuple(sys.nvec[k2] - Q))
                if a is not None and b is not None:
                    lam += P[a, k2] * P[b, k1]
        for k2 in range(M):
            b = where.get(tuple(sys.nvec[k2] - Q))
            if b is not None:
                g2 += P[b, k2]
        E2 += (2.0 * np.pi / (sys.omega * np.sum(((2 * np.pi / sys.L) * np.array(Q)) ** 2))) * \
            (4.0 * g1 * g2 - 2.0 * lam)
    N = 2.0 * np.trace(P)
    return dict(E1=E1, E2=E2, E=E1 + E2 + sys.E_M, N=N)


def density_correlation(sys, G):
    """Local estimator of <rho(Q) rho(-Q)> for every momentum transfer Q (both spins), whose
    ratio to N is the static structure factor S(Q) of Sec. "Results" (structure factor
    section).  Wick's theorem with P = I - G^T (P_ij = <a^+_i a_j> per spin):
      <rho(Q) rho(-Q)> = 4 r_Q r_{-Q} + 2 (n_Q - Lambda_Q),
    r_Q = sum_K P_{K+Q,K} (per spin), n_Q = sum_{K: K, K+Q in basis} P_{K+Q,K+Q} (the contraction
    of a_K with a^+_{K}), Lambda_Q the exchange sum of local_energy."""
    P = np.eye(sys.M) - G.T
    rho = np.array([P[sys.pairs[q]].sum() for q in range(sys.NQ)], dtype=np.complex128)
    out = np.empty(sys.NQ, dtype=np.complex128)
    for q in range(sys.NQ):
        p, r = sys.pairs[q]
        lam = np.sum(P[np.ix_(p, p)] * P[np.ix_(r, r)].T)
        nq = np.sum(P[p, p])
        out[q] = 4.0 * rho[q] * rho[sys.neg[q]] + 2.0 * (nq - lam)
    return out
