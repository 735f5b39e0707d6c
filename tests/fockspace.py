"""Fock-space brute force for tiny plane-wave bases (test infrastructure).

Builds second-quantised operators by the Jordan-Wigner construction and the
UEG Hamiltonian straight from its definition in the paper's Sec. "Uniform
Electron Gas" (kinetic term, normal-ordered Coulomb interaction over all
momentum transfers inside the basis, Madelung constant).  Used only to pin the
oracle: traces, determinants, Wick energies and the sum-of-squares identity.
"""
import numpy as np
import scipy.sparse as sp
import scipy.linalg as sla


def annihilators(nmodes, sparse=False):
    """Jordan-Wigner annihilation operators a_0 .. a_{n-1} on 2^n states."""
    a = np.array([[0.0, 1.0], [0.0, 0.0]])
    Z = np.diag([1.0, -1.0])
    I2 = np.eye(2)
    kron = (lambda x, y: sp.kron(x, y, format="csr")) if sparse else np.kron
    ops = []
    for p in range(nmodes):
        mats = [Z] * p + [a] + [I2] * (nmodes - p - 1)
        op = sp.csr_matrix(mats[0]) if sparse else mats[0]
        for m in mats[1:]:
            op = kron(op, sp.csr_matrix(m) if sparse else m)
        ops.append(op)
    return ops


def lift_one_body(O, a):
    """sum_pq O_pq a^+_p a_q for dense single-spin operators a."""
    M = O.shape[0]
    F = np.zeros_like(a[0], dtype=np.complex128)
    for p in range(M):
        for q in range(M):
            if O[p, q] != 0:
                F = F + O[p, q] * (a[p].conj().T @ a[q])
    return F


def lift_exp_one_body(X, a):
    """Fock operator exp(sum_pq X_pq a^+_p a_q) (dense)."""
    return sla.expm(lift_one_body(X, a))


def same_spin_coulomb(sys, a):
    """(1/2 Omega) sum_{Q!=0} 4pi/Q^2 sum_{K1,K2} a^+_{K1+Q} a^+_{K2-Q} a_{K2} a_{K1}, one spin."""
    where = {tuple(v): i for i, v in enumerate(sys.nvec)}
    dim = a[0].shape[0]
    V = np.zeros((dim, dim), dtype=np.complex128)
    ad = [x.conj().T for x in a]
    for q in range(sys.NQ):
        Q = sys.qvec[q]
        for k1 in range(sys.M):
            i1 = where.get(tuple(sys.nvec[k1] + Q))
            if i1 is None:
                continue
            for k2 in range(sys.M):
                i2 = where.get(tuple(sys.nvec[k2] - Q))
                if i2 is None:
                    continue
                V += 0.5 * sys.vq[q] * (ad[i1] @ ad[i2] @ a[k2] @ a[k1])
    return V


def rho_operator(sys, q, a):
    """rho(Q_q) = sum_K a^+_{K+Q} a_K, one spin."""
    O = np.zeros((sys.M, sys.M))
    O[sys.pairs[q]] = 1.0
    return lift_one_body(O, a)


def two_spin_hamiltonian_sparse(sys, kscale=1.0):
    """H = lambda T + V_ee + E_M on 2M spin-orbitals (mode 2K = K up, 2K+1 = K down), sparse."""
    M = sys.M
    a = annihilators(2 * M, sparse=True)
    ad = [x.T.tocsr() for x in a]
    dim = a[0].shape[0]
    H = sp.csr_matrix((dim, dim))
    for k in range(M):
        for s in range(2):
            H = H + kscale * sys.eps[k] * (ad[2 * k + s] @ a[2 * k + s])
    where = {tuple(v): i for i, v in enumerate(sys.nvec)}
    for q in range(sys.NQ):
        Q = sys.qvec[q]
        for k1 in range(M):
            i1 = where.get(tuple(sys.nvec[k1] + Q))
            if i1 is None:
                continue
            for k2 in range(M):
                i2 = where.get(tuple(sys.nvec[k2] - Q))
                if i2 is None:
                    continue
                for s1 in range(2):
                    for s2 in range(2):
                        H = H + 0.5 * sys.vq[q] * (ad[2 * i1 + s1] @ ad[2 * i2 + s2]
                                                   @ a[2 * k2 + s2] @ a[2 * k1 + s1])
    H = H + sys.E_M * sp.identity(dim, format="csr")
    return H, a


def number_sector(nmodes, n):
    """Indices of the occupation states with n particles (bit p = occupation of mode p)."""
    idx = []
    for state in range(2 ** nmodes):
        # mode 0 is the most significant kron factor
        occ = [(state >> (nmodes - 1 - p)) & 1 for p in range(nmodes)]
        if sum(occ) == n:
            idx.append(state)
    return np.array(idx)
