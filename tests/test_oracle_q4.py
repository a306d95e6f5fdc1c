"""CPU pins of the RCCSDTQ oracle (oracle/rccsdtq.py) against what the
mathematics fixes, independent of its own formulas:

* brute force at arbitrary amplitudes: with every rank non-zero (T1 dressing
  included, non-diagonal Fock matrix), R1 and R2 equal the spin-orbital
  residuals r_{i alpha}^{a alpha} and r_{i alpha j beta}^{a alpha b beta},
  and the spin-free R3 and R4, mapped to spin orbitals by M (antisymmetrised
  over spin-matched virtual columns), equal the spin-orbital triples and
  quadruples residuals <Phi_mu| exp(-T) H exp(T) |Phi_0> of the determinant
  space (Appendix "Coupled-cluster theory");
* dropping any one of the fifteen R4 terms, or any T4 term of R2 or R3,
  breaks that pin;
* the R4 projector of Eq. T4ortho: its character form equals the printed
  polynomial in the sum of transpositions, it is idempotent, keeps 14 of the
  24 virtual permutations, and M annihilates what it removes;
* four electrons (o = 2): converged RCCSDTQ is exact (equals FCI);
* six electrons: at converged RCCSDTQ amplitudes the brute-force
  spin-orbital CCSDTQ residual vanishes and the energies agree.
"""

import itertools

import numpy as np
import pytest

import cct_inputs as ci
from oracle import rccsdt as R, rccsdtq as Q4, spinorb as S


def _system(o, v, seed, sigma=0.2, nondiag=True):
    s = ci.make_system(o, v, 2 * (o + v), seed, sigma=sigma)
    f = ci.random_fock(o, v, seed) if nondiag else s["f"]
    return f, R.eri_phys_from_B(s["B"])


def _phys_t4(o, v, rng, scale=0.05):
    t = Q4.perm_sym4(rng.normal(0.0, scale, (o, o, o, o, v, v, v, v))) / 24.0
    return Q4.project_r4(Q4.purify_r4(t))


def _amps(o, v, seed):
    t1, t2, t3 = ci.random_amplitudes(o, v, seed, 0.05, 0.05, 0.05)
    t3 = R.orthogonalize_r3(R.purify_r3(t3))
    return t1, t2, t3, _phys_t4(o, v, np.random.default_rng(seed + 1000))


class Brute:
    def __init__(self, f, V, o):
        self.sysm = S.SpinOrbitalSystem(f, V, o)
        self.excs = self.sysm.excitations(4)
        self.sysm.prepare(self.excs)
        self.rank = np.array([len(I) for I, _ in self.excs])
        self.o, self.v = o, f.shape[0] - o

    def residual(self, t1, t2, t3, t4):
        tso = S.spinfree_to_spinorb(self.excs, self.o, t1, t2, t3, t4)
        return self.sysm.cc_residual(tso)

    def m(self, rank, x):
        """M (spin-free -> spin-orbital) of a rank-`rank` tensor x, restricted
        to the spin-orbital excitations of that rank."""
        o, v = self.o, self.v
        t = [np.zeros((o, v)), np.zeros((o, o, v, v)), np.zeros((o, o, o, v, v, v)), None]
        t[rank - 1] = x
        out = S.spinfree_to_spinorb(self.excs, o, *t)
        return out[self.rank == rank]


def _pin_errors(f, V, o, v, amps, terms=None, drop_r2=False, drop_r3=None):
    t1, t2, t3, t4 = amps
    b = Brute(f, V, o)
    _, rso = b.residual(t1, t2, t3, t4)
    r1, r2, r3, r4 = Q4.residuals(f, V, t1, t2, t3, t4, o, terms=terms)
    b1, b2, _ = S.spinorb_to_spinfree(b.excs, rso, o, v)
    e1 = np.abs(r1 - b1).max()
    e2 = np.abs(r2 - b2).max()
    e3 = np.abs(b.m(3, r3) - rso[b.rank == 3]).max()
    e4 = np.abs(b.m(4, r4) - rso[b.rank == 4]).max()
    return (e1, e2, e3, e4), np.abs(rso[b.rank == 4]).max()


@pytest.mark.parametrize("o,v,seed", [(2, 2, 1), (2, 3, 2), (3, 2, 3), (3, 3, 4)])
def test_residuals_match_spin_orbital_bruteforce(o, v, seed):
    f, V = _system(o, v, seed)
    amps = _amps(o, v, seed)
    errs, scale = _pin_errors(f, V, o, v, amps)
    assert scale > 1e-3
    for e in errs:
        assert e < 1e-13, errs


@pytest.mark.parametrize("term", Q4.R4_TERMS)
def test_dropping_an_r4_term_breaks_the_pin(term):
    # v = 3: with two virtual orbitals some terms lie wholly in the null space
    o, v, seed = 3, 3, 3
    f, V = _system(o, v, seed)
    amps = _amps(o, v, seed)
    keep = tuple(t for t in Q4.R4_TERMS if t != term)
    errs, _ = _pin_errors(f, V, o, v, amps, terms=keep)
    assert errs[3] > 1e-6, (term, errs)


def test_t4_feedback_into_r2_and_r3_is_pinned():
    """With T4 alone non-zero (T1 = T2 = T3 = 0), R2 and R3 are exactly the
    T4 terms of the RCCSDTQ appendix; scaling them breaks the pin."""
    o, v, seed = 3, 2, 4
    f, V = _system(o, v, seed, nondiag=False)
    t1, t2, t3, t4 = _amps(o, v, seed)
    z = (np.zeros_like(t1), np.zeros_like(t2), np.zeros_like(t3))
    b = Brute(f, V, o)
    _, rso = b.residual(*z, t4)
    r1, r2, r3, r4 = Q4.residuals(f, V, *z, t4, o)
    r1_0, r2_0, r3_0 = R.residuals(f, V, *z, o)
    b1, b2, _ = S.spinorb_to_spinfree(b.excs, rso, o, v)
    assert np.abs(r2 - b2).max() < 1e-13
    assert np.abs(b.m(3, r3) - rso[b.rank == 3]).max() < 1e-13
    d2, d3 = r2 - r2_0, r3 - r3_0
    assert np.abs(d2).max() > 1e-4 and np.abs(b.m(3, d3)).max() > 1e-4
    assert np.abs(r2_0 + 0.9 * d2 - b2).max() > 1e-6
    assert np.abs(b.m(3, r3_0 + 0.9 * d3) - rso[b.rank == 3]).max() > 1e-6


def test_r4_projector():
    rng = np.random.default_rng(5)
    o, v = 2, 4
    x = Q4.perm_sym4(rng.normal(size=(o, o, o, o, v, v, v, v)))
    p = Q4.project_r4(x)
    assert np.abs(p - Q4.project_r4_polynomial(x)).max() < 1e-12 * np.abs(x).max()
    assert np.abs(Q4.project_r4(p) - p).max() < 1e-12 * np.abs(x).max()
    # on one virtual orbit of four distinct labels the projector has rank 14 of 24
    perms = list(itertools.permutations(range(4)))
    Pm = np.zeros((24, 24))
    for c, q in enumerate(perms):
        e = np.zeros((1, 1, 1, 1, 4, 4, 4, 4))
        e[(0, 0, 0, 0) + q] = 1.0
        y = Q4.project_r4(e)
        for r, w in enumerate(perms):
            Pm[r, c] = y[(0, 0, 0, 0) + w]
    assert abs(np.trace(Pm) - 14.0) < 1e-12
    assert np.linalg.matrix_rank(Pm) == 14
    # M maps the removed (redundant) part to zero
    f, V = _system(3, 2, 6)
    b = Brute(f, V, 3)
    t4 = Q4.perm_sym4(np.random.default_rng(7).normal(size=(3, 3, 3, 3, 2, 2, 2, 2)))
    t4 = Q4.purify_r4(t4)
    null = t4 - Q4.project_r4(t4)
    assert np.abs(null).max() > 1e-3
    assert np.abs(b.m(4, null)).max() < 1e-12


def test_four_electrons_rccsdtq_is_exact():
    """o = 2 (four electrons): CCSDTQ is full CI."""
    o, v = 2, 3
    f, V = _system(o, v, 8, sigma=0.15, nondiag=False)
    e, *_, it, conv = Q4.solve(f, V, o, tol=1e-11, max_iter=400)
    assert conv
    sysm = S.SpinOrbitalSystem(f, V, o)
    efci, _ = sysm.fci_vector()
    assert abs(e - (efci - sysm.hf_energy())) < 1e-10


def test_six_electrons_two_virtuals_rccsdtq_is_exact():
    """o = 3, v = 2: four virtual spin orbitals allow at most quadruple
    excitations, so CCSDTQ is full CI here too."""
    o, v = 3, 2
    f, V = _system(o, v, 9, sigma=0.15, nondiag=False)
    e, *_, it, conv = Q4.solve(f, V, o, tol=1e-11, max_iter=400)
    assert conv
    sysm = S.SpinOrbitalSystem(f, V, o)
    efci, _ = sysm.fci_vector()
    assert abs(e - (efci - sysm.hf_energy())) < 1e-10


def test_six_electrons_converged_amplitudes_solve_bruteforce_ccsdtq():
    """o = 3, v = 3: at converged RCCSDTQ amplitudes every spin-orbital
    residual of rank 1..4 vanishes and the brute-force energy is the same;
    CCSDTQ is not exact here (quintuples and sextuples exist)."""
    o, v = 3, 3
    f, V = _system(o, v, 10, sigma=0.15, nondiag=False)
    e, t1, t2, t3, t4, it, conv = Q4.solve(f, V, o, tol=1e-12, max_iter=400)
    assert conv
    b = Brute(f, V, o)
    etot, rso = b.residual(t1, t2, t3, t4)
    assert np.abs(rso).max() < 1e-10
    assert abs((etot - b.sysm.hf_energy()) - e) < 1e-11
    efci, _ = b.sysm.fci_vector()
    assert abs(e - (efci - b.sysm.hf_energy())) > 1e-7
