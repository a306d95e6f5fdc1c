"""Pins of the (Q) oracle (oracle/rccsdt_q.py) against what the mathematics
fixes, independent of its own formulas:

* brute force: the spin-free E_(Q) equals the spin-orbital CCSDT(Q) energy
  evaluated with explicit operators in determinant space
  (sum_Q <Q|H_N(T2+T3)|0> <Q|H_N T3 + 1/2 (H_N T2^2)_C|0> / D_Q), at random
  physical amplitudes and at converged RCCSDT amplitudes;
* planted mistakes in each term, and in the spin summation, break that pin;
* two electrons (o = 1) have no quadruples: E_(Q) = 0;
* the fully spin-summed amplitude vanishes when three occupied labels are
  equal (one spatial orbital holds two electrons) and is invariant under
  simultaneous column permutations, so that E_(Q) = sum (X + V) . tchk, the
  form the GPU path evaluates.
"""

import numpy as np
import pytest

import cct_inputs as ci
from oracle import rccsdt as R, rccsdt_q as Q, spinorb as S


def _system(o, v, seed, sigma=0.2):
    s = ci.make_system(o, v, 2 * (o + v), seed, sigma=sigma)
    return s["f"], R.eri_phys_from_B(s["B"])


def _amps(o, v, seed):
    _, t2, t3 = ci.random_amplitudes(o, v, seed, 0.05, 0.05, 0.05)
    return t2, R.orthogonalize_r3(R.purify_r3(t3))


def _brute(f, V, o, v, t2, t3):
    sysm = S.SpinOrbitalSystem(f, V, o)
    sysm.prepare(sysm.excitations(4))
    tso = S.spinfree_to_spinorb(sysm.excs, o, np.zeros((o, v)), t2, t3)
    return sysm.q_correction(tso, np.diag(f))


@pytest.mark.parametrize("o,v,seed", [(2, 2, 1), (2, 3, 3), (3, 2, 2)])
def test_energy_q_matches_spin_orbital_bruteforce(o, v, seed):
    f, V = _system(o, v, seed)
    t2, t3 = _amps(o, v, seed + 1)
    eb = _brute(f, V, o, v, t2, t3)
    assert abs(eb) > 1e-4
    assert abs(Q.energy_q(f, V, t2, t3, o) - eb) < 1e-14


def test_energy_q_at_converged_rccsdt_matches_bruteforce():
    o, v = 2, 3
    f, V = _system(o, v, 12)
    e, t1, t2, t3, _, conv = R.solve(f, V, o, tol=1e-12, max_iter=300)
    assert conv
    eb = _brute(f, V, o, v, t2, t3)
    assert abs(eb) > 1e-6
    assert abs(Q.energy_q(f, V, t2, t3, o) - eb) < 1e-14


def _energy_from_parts(f, V, X, Y, Vt, o, spin_sum):
    t4 = Q.perm_sym4(X + Y) / Q.denominators4(f, o)
    z = Q.perm_sym4(X + Vt)
    return float(np.einsum("ijklabcd,ijklabcd->", z, spin_sum(t4)) / 24.0)


def _bad_spin_sum(t4):
    def swap(x, p, q):
        ax = list(range(8))
        ax[4 + p], ax[4 + q] = ax[4 + q], ax[4 + p]
        return x.transpose(ax)
    u1 = 2 * t4 - swap(t4, 0, 1) - swap(t4, 0, 2) - swap(t4, 0, 3)
    u2 = 2 * u1 - swap(u1, 1, 2) - swap(u1, 1, 3)
    return 2 * (2 * u2 - swap(u2, 1, 3))          # wrong pair in the last factor


@pytest.mark.parametrize("mistake", ["X1", "X2", "Y1", "Y2", "V", "V_sign", "Wo_ring1", "Wo_ring2", "Wo_hole",
                                     "spin_sum"])
def test_planted_mistake_breaks_the_bruteforce_pin(mistake):
    o, v, seed = 2, 3, 3
    f, V = _system(o, v, seed)
    t2, t3 = _amps(o, v, seed + 1)
    eb = _brute(f, V, o, v, t2, t3)
    O, Vs = slice(0, o), slice(o, None)
    X1 = 0.5 * np.einsum("abej,iklecd->ijklabcd", V[Vs, Vs, Vs, O], t3)
    X2 = -0.5 * np.einsum("amij,mklbcd->ijklabcd", V[Vs, O, O, O], t3)
    Y1 = 0.5 * np.einsum("ejkabc,iled->ijklabcd", Q.wbar_vvvo(V, t2, o), t2)
    g = [np.einsum("maei,jkbe->ijkabm", V[O, Vs, Vs, O], t2),
         np.einsum("make,jibe->ijkabm", V[O, Vs, O, Vs], t2),
         -0.5 * np.einsum("mnki,njab->ijkabm", V[O, O, O, O], t2)]

    def y2(parts):
        w = sum(parts)
        return -0.5 * np.einsum("ijkabm,mlcd->ijklabcd", w + w.transpose(1, 0, 2, 4, 3, 5), t2)

    Vt = Q.v_term(V, t2, o)
    X, Y, spin = X1 + X2, Y1 + y2(g), Q.spin_sum4
    assert abs(_energy_from_parts(f, V, X, Y, Vt, o, spin) - eb) < 1e-14
    if mistake == "X1":
        X = X2
    elif mistake == "X2":
        X = X1
    elif mistake == "Y1":
        Y = y2(g)
    elif mistake == "Y2":
        Y = Y1
    elif mistake == "V":
        Vt = 0.0 * Vt
    elif mistake == "V_sign":
        Vt = -Vt
    elif mistake.startswith("Wo_"):
        drop = {"Wo_ring1": 0, "Wo_ring2": 1, "Wo_hole": 2}[mistake]
        Y = Y1 + y2([x for n, x in enumerate(g) if n != drop])
    elif mistake == "spin_sum":
        spin = _bad_spin_sum
    assert abs(_energy_from_parts(f, V, X, Y, Vt, o, spin) - eb) > 1e-6


@pytest.mark.parametrize("v", [2, 3, 4])
def test_two_electrons_have_no_quadruples(v):
    f, V = _system(1, v, 5)
    t2, t3 = _amps(1, v, 6)
    assert abs(Q.energy_q(f, V, t2, t3, 1)) < 1e-30


def test_spin_summed_quadruples_symmetry_and_vanishing_triples():
    o, v = 3, 3
    f, V = _system(o, v, 7)
    t2, t3 = _amps(o, v, 8)
    t4, z = Q.quadruples(f, V, t2, t3, o)
    U = Q.spin_sum4(t4)
    assert np.abs(U).max() > 1e-3
    for p in Q.PERMS4:
        assert np.abs(U - U.transpose(*p, *(4 + q for q in p))).max() < 1e-15
    for i in range(o):
        for l in range(o):
            assert np.abs(U[i, i, i, l]).max() < 1e-15
    A = Q.x_term(V, t3, o) + Q.v_term(V, t2, o)
    e_paper = np.einsum("ijklabcd,ijklabcd->", z, U) / 24.0
    assert abs(np.einsum("ijklabcd,ijklabcd->", A, U) - e_paper) < 1e-15


@pytest.mark.parametrize("o,v,seed", [(3, 5, 2), (4, 6, 4)])
def test_task_energy_matches_full_tensor_split(o, v, seed):
    """The one-tuple-at-a-time oracle (for sizes where o^4 v^4 does not fit)
    equals the full-tensor sum over each task's distinct orderings of
    (X + V) . tchk, and the tasks add up to E_(Q)."""
    import itertools
    f, V = _system(o, v, seed, sigma=0.1)
    t2, t3 = _amps(o, v, seed + 1)
    t4, _ = Q.quadruples(f, V, t2, t3, o)
    U = Q.spin_sum4(t4)
    A = Q.x_term(V, t3, o) + Q.v_term(V, t2, o)
    total = 0.0
    for i in range(o):
        for j in range(i, o):
            for k in range(j, o):
                for l in range(k, o):
                    ref = sum(float(np.sum(A[q] * U[q])) for q in set(itertools.permutations((i, j, k, l))))
                    got = Q.task_energy(f, V, t2, t3, o, (i, j, k, l))
                    assert abs(got - ref) < 1e-15
                    total += got
    assert abs(total - Q.energy_q(f, V, t2, t3, o)) < 1e-14


# --- the virtual-tuple (ABC) order and the alternative intermediates ---------

@pytest.mark.parametrize("o,v,seed", [(2, 3, 21), (3, 4, 22)])
def test_alternative_intermediates_give_the_same_residual(o, v, seed):
    """Eq. q_w_alter moves terms between the two Wbar intermediates: Y changes
    element by element, its 24-permutation sum (the residual) does not; the
    energy with the alternative Y equals the brute-force-pinned one."""
    f, V = _system(o, v, seed)
    t2, t3 = _amps(o, v, seed + 1)
    Y, Ya = Q.y_term(V, t2, o), Q.y_term_alt(V, t2, o)
    assert np.abs(Y - Ya).max() > 1e-4
    PY, PYa = Q.perm_sym4(Y), Q.perm_sym4(Ya)
    assert np.abs(PY - PYa).max() <= 1e-14 * max(1.0, np.abs(PY).max())
    X, Vt = Q.x_term(V, t3, o), Q.v_term(V, t2, o)
    e_alt = _energy_from_parts(f, V, X, Ya, Vt, o, Q.spin_sum4)
    assert abs(e_alt - Q.energy_q(f, V, t2, t3, o)) < 1e-14
    # a sign slip in either moved term is caught
    O, Vs = slice(0, o), slice(o, None)
    bad = Q.wbar_vvvo_alt(V, t2, o)
    g = np.einsum("mbej,mkac->ejkabc", V[O, Vs, Vs, O], t2)
    bad = bad + 2 * (g + g.transpose(0, 2, 1, 3, 5, 4))
    Yb = 0.5 * np.einsum("ejkabc,iled->ijklabcd", bad, t2) - 0.5 * np.einsum(
        "ijkabm,mlcd->ijklabcd", Q.wbar_vooo_alt(V, t2, o), t2)
    assert np.abs(Q.perm_sym4(Yb) - PY).max() > 1e-6


@pytest.mark.parametrize("o,v,seed", [(2, 3, 23), (3, 4, 24), (2, 5, 25)])
def test_virtual_tuple_order_sums_to_the_energy(o, v, seed):
    """Eq. ener-pt-q-abc: the sum over a <= b <= c <= d with the ordering
    multiplicities is E_(Q); tuples with three equal virtual labels give 0
    (the fully spin-summed amplitude vanishes there, as for three equal
    occupied labels); the one-tuple evaluation (alternative intermediates,
    o^4 arrays, the spin summation applied to the occupied axes) reproduces
    every tuple's share."""
    f, V = _system(o, v, seed)
    t2, t3 = _amps(o, v, seed + 1)
    e = Q.energy_q(f, V, t2, t3, o)
    total, parts = Q.energy_q_by_virtual_tuples(f, V, t2, t3, o)
    assert abs(total - e) < 1e-14
    for (a, b, c, d), x in parts.items():
        if a == b == c or b == c == d:
            assert abs(x) < 1e-15
    s = 0.0
    for t, x in parts.items():
        y = Q.virtual_task_energy(f, V, t2, t3, o, t)
        assert abs(y - x) < 1e-14, (t, x, y)
        s += y
    assert abs(s - e) < 1e-14 and abs(e) > 1e-5
