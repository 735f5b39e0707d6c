"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds workload parameters and a random-number recipe only; it does
none of the method's arithmetic.  The auxiliary fields of the Hubbard-Stratonovich
transform are iid standard normal (Sec. "Finite-Temperature AFQMC", the HS
transform); here each momentum transfer Q of a slice carries one complex128
number whose real part is the field of A(Q) and whose imaginary part is the
field of B(Q) (Sec. "Uniform Electron Gas", the sum-of-squares form).

Recipe: walker w of a workload with seed s draws its fields from
numpy.random.Generator(PCG64(SeedSequence([s, w]))) as standard_normal of shape
(n_slices, n_q, 2), viewed as complex128 (n_slices, n_q).  Drawing per walker
lets a test take any subset of walkers without drawing the rest.
"""
import numpy as np

# Workload parameters (electron number, Wigner-Seitz radius, reduced temperature
# Theta = T/T_F, plane-wave cutoff |n|^2 <= nmax2, nominal time step in Hartree^-1,
# stabilisation interval in slices, walker count).  The uneven batch lists four
# systems that run together.
WORKLOADS = {
    "ueg_n14_m19": dict(systems=[dict(n_elec=14, rs=1.0, theta=0.5, nmax2=2, dtau=0.05,
                                      stab_every=5, walkers=64)], seed=122281),
    "ueg_n66_m171": dict(systems=[dict(n_elec=66, rs=1.0, theta=0.125, nmax2=11, dtau=0.025,
                                       stab_every=10, walkers=256)], seed=122282),
    "ueg_n38_m123": dict(systems=[dict(n_elec=38, rs=2.0, theta=0.25, nmax2=9, dtau=0.05,
                                       stab_every=10, walkers=128)], seed=122283),
    "ueg_uneven4": dict(systems=[
        dict(n_elec=14, rs=0.5, theta=0.0625, nmax2=2, dtau=0.05, stab_every=10, walkers=171),
        dict(n_elec=38, rs=1.0, theta=0.125, nmax2=5, dtau=0.05, stab_every=10, walkers=171),
        dict(n_elec=54, rs=2.0, theta=0.25, nmax2=9, dtau=0.05, stab_every=10, walkers=85),
        dict(n_elec=66, rs=4.0, theta=0.5, nmax2=11, dtau=0.05, stab_every=10, walkers=85),
    ], seed=122284),
    "ueg_n114_m485": dict(systems=[dict(n_elec=114, rs=0.5, theta=0.0625, nmax2=24, dtau=0.02,
                                        stab_every=8, walkers=512)], seed=122285),
}


def system_seed(workload, system_index):
    """Seed of one system of a workload: the workload seed plus 1000 per system index."""
    return int(WORKLOADS[workload]["seed"]) + 1000 * int(system_index)


def walker_rng(seed, walker):
    """The generator of one walker: PCG64 seeded by the pair (seed, walker)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(walker)])))


def walker_fields(seed, walker, n_slices, n_q):
    """complex128 array (n_slices, n_q) of iid N(0,1) real and imaginary parts."""
    g = walker_rng(seed, walker)
    x = g.standard_normal(size=(n_slices, n_q, 2))
    return np.ascontiguousarray(x).view(np.complex128)[..., 0]


def fields(seed, walkers, n_slices, n_q, out=None):
    """complex128 array (len(walkers), n_slices, n_q); walkers is an int or a list of ids."""
    ids = range(walkers) if isinstance(walkers, (int, np.integer)) else list(walkers)
    ids = list(ids)
    if out is None:
        out = np.empty((len(ids), n_slices, n_q), dtype=np.complex128)
    for i, w in enumerate(ids):
        out[i] = walker_fields(seed, w, n_slices, n_q)
    return out
