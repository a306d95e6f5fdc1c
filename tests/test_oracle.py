"""CPU pins of the FP64 oracle against things other than itself: brute-force
determinant-space CC and FCI, closed forms, special cases and invariants.

A plausible transcription mistake in any residual term (a dropped term, a
wrong sign, index or operand order) changes R1, R2 or the physical part of R3
at generic amplitudes, which the brute-force residual pin catches; the
planted-mistake test below checks that this is so for every R3 term.
"""

import itertools
import os

import numpy as np
import pytest

import cct_inputs as ci
from oracle import counts, rccsdt as R, spinorb as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return [float(x) for x in fh.read().split("\n") if x and not x.startswith("#")]


def _tiny(o, v, seed, sigma=0.2):
    s = ci.make_system(o, v, 2 * (o + v), seed, sigma=sigma)
    V = R.eri_phys_from_B(s["B"])
    f = ci.random_fock(o, v, seed)
    return f, V


def _brute_residuals(f, V, o, v, t1, t2, t3):
    sysm = S.SpinOrbitalSystem(f, V, o)
    excs = sysm.excitations(3)
    sysm.prepare(excs)
    tso = S.spinfree_to_spinorb(excs, o, t1, t2, t3)
    e, r = sysm.cc_residual(tso)
    b1, b2, b3 = S.spinorb_to_spinfree(excs, r, o, v)
    return e - sysm.hf_energy(), b1, b2, b3


# ---------------------------------------------------------------------------
# input generator
# ---------------------------------------------------------------------------

def test_generator_anchor_mp2():
    (anchor,) = _read_golden("mp2_anchor_o4v20_seed1.txt")
    s = ci.make_system(4, 20, 48, 1)
    V = R.eri_phys_from_B(s["B"])
    t1, t2, _ = R.mp2_guess(s["f"], V, 4)
    assert abs(R.energy(s["f"], V, t1, t2, 4) - anchor) < 1e-13


def test_generator_symmetries():
    s = ci.make_system(3, 5, 16, 7)
    assert np.array_equal(s["B"], s["B"].transpose(0, 2, 1))
    t3p = ci.random_t3_packed(3, 4, 9)
    for idx, (i, j, k) in enumerate(ci.packed_triples(3)):
        b = t3p[idx]
        if i == j:
            assert np.array_equal(b, b.transpose(1, 0, 2))
        if j == k:
            assert np.array_equal(b, b.transpose(0, 2, 1))


# ---------------------------------------------------------------------------
# brute-force machinery against textbook identities
# ---------------------------------------------------------------------------

def test_bruteforce_ccsdt_three_electrons_equals_fci():
    """Full-rank projective CC reproduces FCI: with 3 electrons CCSDT is exact.
    Amplitudes from the FCI vector's cluster decomposition make every
    brute-force residual vanish and give the FCI energy."""
    f, V = _tiny(2, 2, 5, sigma=0.3)
    sysm = S.SpinOrbitalSystem(f, V, 2, ref_occ=[0, 1, 2])
    efci, c = sysm.fci_vector()
    sysm.prepare(sysm.excitations(3))
    t = sysm.amplitudes_from_ci(c)
    e, r = sysm.cc_residual(t)
    assert abs(e - efci) < 1e-12
    assert np.linalg.norm(r) < 1e-12


def test_bruteforce_ccsd_two_electrons_equals_fci():
    s = ci.make_system(1, 3, 8, 6, sigma=0.3)
    V = R.eri_phys_from_B(s["B"])
    sysm = S.SpinOrbitalSystem(s["f"], V, 1)
    ecc, _, conv = S.solve_cc(sysm, 2)
    assert conv
    assert abs(ecc - (sysm.fci() - sysm.hf_energy())) < 1e-11


# ---------------------------------------------------------------------------
# restricted oracle pins
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("v", [2, 3, 4])
def test_two_electrons_rccsd_rccsdt_fci(v):
    """o = 1: every T3 block is an i=j=k block (purified), so RCCSDT = RCCSD,
    and CCSD is exact for two electrons."""
    s = ci.make_system(1, v, 2 * (1 + v), 20 + v, sigma=0.3)
    V = R.eri_phys_from_B(s["B"])
    sysm = S.SpinOrbitalSystem(s["f"], V, 1)
    efci = sysm.fci() - sysm.hf_energy()
    e_sd, *_, conv1 = R.solve(s["f"], V, 1, triples=False, tol=1e-12)
    e_sdt, *_, conv2 = R.solve(s["f"], V, 1, triples=True, tol=1e-12)
    assert conv1 and conv2
    assert abs(e_sd - efci) < 1e-10
    assert abs(e_sdt - efci) < 1e-10


@pytest.mark.parametrize("o,v,seed", [(2, 2, 1), (2, 3, 3), (3, 2, 2), (3, 3, 4)])
def test_residuals_match_bruteforce(o, v, seed):
    """At generic amplitudes (nonzero T1, T2, physical T3, non-diagonal f):
    r1 = r_{i alpha}^{a alpha}, r2 = r_{i alpha j beta}^{a alpha b beta}, and the
    post-processed R3 equals L(r3 spin-orbital); the energy expression equals
    <Phi_0|Hbar|Phi_0> - E_HF."""
    f, V = _tiny(o, v, seed)
    t1, t2, t3 = ci.random_amplitudes(o, v, seed + 1, 0.05, 0.05, 0.05)
    t3 = R.orthogonalize_r3(R.purify_r3(t3))
    r1, r2, r3 = R.residuals(f, V, t1, t2, t3, o)
    r3 = R.postprocess_r3(r3)
    ebf, b1, b2, b3 = _brute_residuals(f, V, o, v, t1, t2, t3)
    assert abs(R.energy(f, V, t1, t2, o) - ebf) < 1e-13
    assert np.abs(r1 - b1).max() < 1e-13
    assert np.abs(r2 - b2).max() < 1e-13
    assert np.abs(r3 - b3).max() < 1e-13
    assert np.abs(b3).max() > 1e-2


@pytest.mark.parametrize("term", R.R3_TERMS)
def test_planted_mistake_is_caught(term):
    """Dropping any single R3 term breaks the brute-force residual pin."""
    o, v, seed = 2, 3, 3
    f, V = _tiny(o, v, seed)
    t1, t2, t3 = ci.random_amplitudes(o, v, seed + 1, 0.05, 0.05, 0.05)
    t3 = R.orthogonalize_r3(R.purify_r3(t3))
    keep = tuple(x for x in R.R3_TERMS if x != term)
    r3 = R.postprocess_r3(R.residuals(f, V, t1, t2, t3, o, terms=keep)[2])
    _, _, _, b3 = _brute_residuals(f, V, o, v, t1, t2, t3)
    assert np.abs(r3 - b3).max() > 1e-6


def test_null_space_component_of_t3_is_inert():
    o, v, seed = 2, 3, 3
    f, V = _tiny(o, v, seed)
    t1, t2, t3 = ci.random_amplitudes(o, v, seed + 1, 0.05, 0.05, 0.05)
    t3p = R.orthogonalize_r3(R.purify_r3(t3))
    a = R.postprocess_r3(R.residuals(f, V, t1, t2, t3, o)[2])
    b = R.postprocess_r3(R.residuals(f, V, t1, t2, t3p, o)[2])
    assert np.abs(a - b).max() < 1e-14


@pytest.mark.parametrize("o,v,seed", [(2, 2, 11), (2, 3, 12), (3, 2, 13)])
def test_converged_rccsdt_is_spin_orbital_ccsdt(o, v, seed):
    """The converged spin-free amplitudes, mapped to spin orbitals, solve the
    brute-force CCSDT equations and give the same energy."""
    f, V = _tiny(o, v, seed)
    e, t1, t2, t3, _, conv = R.solve(f, V, o, tol=1e-12, max_iter=300)
    assert conv
    ebf, b1, b2, b3 = _brute_residuals(f, V, o, v, t1, t2, t3)
    sysm = S.SpinOrbitalSystem(f, V, o)
    sysm.prepare(sysm.excitations(3))
    tso = S.spinfree_to_spinorb(sysm.excs, o, t1, t2, t3)
    _, r = sysm.cc_residual(tso)
    assert np.abs(r).max() < 1e-10
    assert abs(e - ebf) < 1e-11


# ---------------------------------------------------------------------------
# closed forms and special cases
# ---------------------------------------------------------------------------

def test_triples_overlap_eigenvalues():
    """S3 overlap m(rho) = sgn(rho) 2^{cycles(rho)}: eigenvalues 0, 6 (x4), 24;
    the null vector is the fully symmetric one."""
    perms = list(itertools.permutations(range(3)))

    def compose(p, q):
        return tuple(p[q[x]] for x in range(3))

    def inverse(p):
        inv = [0] * 3
        for a, b in enumerate(p):
            inv[b] = a
        return tuple(inv)

    def cycles(p):
        seen, c = set(), 0
        for s in range(3):
            if s not in seen:
                c += 1
                x = s
                while x not in seen:
                    seen.add(x)
                    x = p[x]
        return c

    M = np.array([[S._perm_sign(compose(inverse(p), q)) * 2.0 ** cycles(compose(inverse(p), q)) for q in perms]
                  for p in perms])
    w, U = np.linalg.eigh(M)
    assert np.allclose(sorted(w), [0, 6, 6, 6, 6, 24])
    null = U[:, np.argmin(np.abs(w))]
    assert np.allclose(np.abs(null), 1 / np.sqrt(6))


def test_L_after_M_is_orthogonal_projector():
    """L(M(t3)) = (1 - Pi_[3]) t3 for column-symmetric t3."""
    o, v = 3, 3
    f, V = _tiny(o, v, 1)
    _, _, t3 = ci.random_amplitudes(o, v, 5, 0.1, 0.1, 0.1)
    t3 = R.purify_r3(t3)
    sysm = S.SpinOrbitalSystem(f, V, o)
    excs = sysm.excitations(3)
    tso = S.spinfree_to_spinorb(excs, o, np.zeros((o, v)), np.zeros((o, o, v, v)), t3)
    _, _, back = S.spinorb_to_spinfree(excs, tso, o, v)
    assert np.abs(back - R.orthogonalize_r3(t3)).max() < 1e-15


def test_dressing_identity_at_zero_t1():
    f, V = _tiny(2, 3, 8)
    ft, Vt = R.dress(f, V, np.zeros((2, 3)))
    assert np.abs(ft - f).max() == 0.0
    assert np.abs(Vt - V).max() < 1e-16


def test_diagonal_fock_term_gives_minus_denominator():
    """With V = 0, T1 = T2 = 0 and diagonal f, R3 = -eps_ijk^abc t3 (each
    column reaches the first position twice among the six permutations)."""
    o, v = 3, 3
    f = ci.make_system(o, v, 2, 3)["f"]
    V = np.zeros((o + v,) * 4)
    _, _, t3 = ci.random_amplitudes(o, v, 2)
    _, _, r3 = R.residuals(f, V, np.zeros((o, v)), np.zeros((o, o, v, v)), t3, o)
    d3 = R.denominators(f, o)[2]
    assert np.abs(r3 + d3 * t3).max() < 1e-15


def test_r3_invariants():
    o, v = 3, 4
    f, V = _tiny(o, v, 9, sigma=0.1)
    t1, t2, t3 = ci.random_amplitudes(o, v, 10)
    r3 = R.residuals(f, V, t1, t2, t3, o)[2]
    assert np.abs(r3 - r3.transpose(1, 0, 2, 4, 3, 5)).max() < 1e-15
    assert np.abs(r3 - r3.transpose(2, 1, 0, 5, 4, 3)).max() < 1e-15
    p = R.postprocess_r3(r3)
    s = sum(p.transpose(0, 1, 2, 3 + a, 3 + b, 3 + c) for a, b, c in itertools.permutations(range(3)))
    assert np.abs(s).max() < 1e-15
    for i in range(o):
        assert not np.any(p[i, i, i])


def test_pack_unpack_roundtrip():
    o, v = 4, 3
    _, _, t3 = ci.random_amplitudes(o, v, 3)
    assert np.abs(R.unpack_t3(R.pack_t3(t3), o) - t3).max() < 1e-16
    t3p = ci.random_t3_packed(o, v, 4)
    assert np.array_equal(R.pack_t3(R.unpack_t3(t3p, o)), t3p)


def test_mac_counts_reduce_to_paper_leading_terms():
    o, v = 400, 4000
    exact = counts.r3_macs_total(o, v)
    lead = counts.leading_asymptotic(o, v)
    assert abs(exact / lead - 1.0) < 0.02
    assert counts.r3_macs_total(4, 20) == 387840000
    assert abs(counts.r3_macs_total(20, 180) - 1.288e15) / 1.288e15 < 1e-3


def test_block_oracle_matches_full_oracle_pp():
    """oracle.blocks (used where the full tensor does not fit) reproduces the
    full-tensor oracle's particle-particle ladder block by block."""
    from oracle import blocks

    o, v, seed = 3, 5, 17
    s = ci.make_system(o, v, 2 * (o + v), seed, sigma=0.1)
    f = ci.random_fock(o, v, seed)
    V = R.eri_phys_from_B(s["B"])
    t1, t2, _ = ci.random_amplitudes(o, v, seed, 0.03, 0.03, 0.0, triples=False)
    t3p = ci.hashed_t3_packed(o, v, seed, 0.02, threads=2)
    ref = R.pack_t3(R.postprocess_r3(R.residuals(f, V, t1, t2, R.unpack_t3(t3p, o), o, terms=("PP",))[2]))
    W = blocks.w_vvvv(blocks.dressed_factors(s["B"], t1), t2, o)
    for n, ijk in enumerate(ci.packed_triples(o)):
        got = blocks.postprocess_block(blocks.pp_block(W, t3p[n], ijk), ijk)
        assert np.abs(got - ref[n]).max() < 1e-15


def test_block_oracle_local_terms_match_full_oracle():
    """The block forms of the F_vv term and the two T2 drivers reproduce the
    full-tensor oracle's terms (same intermediates) block by block, including
    blocks with repeated occupied indices."""
    from oracle import blocks

    o, v = 3, 5
    rng = np.random.default_rng(23)
    t2 = rng.normal(0, 0.05, (o, o, v, v))
    t2 = 0.5 * (t2 + t2.transpose(1, 0, 3, 2))
    t3p = ci.hashed_t3_packed(o, v, 31, 0.02, threads=2)
    t3 = R.unpack_t3(t3p, o)
    ims = {"Fvv": rng.normal(0, 0.1, (v, v)), "Foo": rng.normal(0, 0.1, (o, o)),
           "Woooo": rng.normal(0, 0.1, (o, o, o, o))}
    ims3 = {"Wvvvo": rng.normal(0, 0.1, (v, v, v, o)), "Wvooo": rng.normal(0, 0.1, (v, o, o, o)),
            "Wbar_ovvo": rng.normal(0, 0.1, (o, v, v, o)), "Wbar_ovov": rng.normal(0, 0.1, (o, v, o, v)),
            "Wvvvv": rng.normal(0, 0.1, (v, v, v, v))}
    parts = R.r3_terms(t2, t3, ims, ims3)
    for name, fn in (("F1", lambda ijk, n: blocks.f1_block(ims["Fvv"], t3p[n], ijk)),
                     ("D1", lambda ijk, n: blocks.d1_block(ims3["Wvvvo"], t2, ijk)),
                     ("D2", lambda ijk, n: blocks.d2_block(ims3["Wvooo"], t2, ijk)),
                     ("PP", lambda ijk, n: blocks.pp_block(ims3["Wvvvv"], t3p[n], ijk))):
        full = R.perm_sym3(parts[name])
        for n, (i, j, k) in enumerate(ci.packed_triples(o)):
            got = fn((i, j, k), n)
            assert np.abs(got - full[i, j, k]).max() < 1e-14, (name, (i, j, k))
    # the combined local sum is the post-processed sum of the four
    full = R.postprocess_r3(sum(R.perm_sym3(parts[k]) for k in ("PP", "F1", "D1", "D2")))
    for n, (i, j, k) in enumerate(ci.packed_triples(o)):
        got = blocks.local_terms_block(ims3["Wvvvv"], ims["Fvv"], ims3["Wvvvo"], ims3["Wvooo"], t2, t3p[n], (i, j, k))
        assert np.abs(got - full[i, j, k]).max() < 1e-14


def test_element_oracle_matches_block_oracle():
    """The element-wise local-terms oracle (W rows on demand, orbit
    post-processing) equals the whole-block oracle on every element of
    several blocks, including repeated occupied and virtual indices."""
    from oracle import blocks

    o, v, naux = 3, 5, 16
    rng = np.random.default_rng(29)
    s = ci.make_system(o, v, naux, 29, sigma=0.1)
    t1, t2, _ = ci.random_amplitudes(o, v, 29, 0.03, 0.03, 0.0, triples=False)
    Bt = blocks.dressed_factors(s["B"], t1)
    Fvv = rng.normal(0, 0.1, (v, v))
    Wvvvo = rng.normal(0, 0.1, (v, v, v, o))
    Wvooo = rng.normal(0, 0.1, (v, o, o, o))
    t3p = ci.hashed_t3_packed(o, v, 30, 0.02, threads=2)
    W = blocks.w_vvvv(Bt, t2, o)
    G = blocks.occ_virt_gram(Bt, o)
    tri = ci.packed_triples(o)
    abcs = [(a, b, c) for a in range(v) for b in range(v) for c in range(v)]
    for n in (0, 1, 4, 5, len(tri) - 1):
        ref = blocks.local_terms_block(W, Fvv, Wvvvo, Wvooo, t2, t3p[n], tri[n])
        got = blocks.local_terms_elements(Bt, t2, Fvv, Wvvvo, Wvooo, t3p[n], tri[n], abcs, G)
        assert np.abs(got - ref.reshape(-1)).max() < 1e-14, tri[n]


def test_hashed_t3_symmetry_and_determinism():
    o, v = 3, 6
    a = ci.hashed_t3_packed(o, v, 5, threads=3)
    b = ci.hashed_t3_packed(o, v, 5, threads=1)
    assert np.array_equal(a, b)
    for idx, (i, j, k) in enumerate(ci.packed_triples(o)):
        blk = a[idx]
        if i == j:
            assert np.array_equal(blk, blk.transpose(1, 0, 2))
        if j == k:
            assert np.array_equal(blk, blk.transpose(0, 2, 1))
    assert abs(a.std() - 0.01 / np.sqrt(3)) < 2e-3


# ---------------------------------------------------------------------------
# DIIS on a T3 subspace (Sec. "Distributed DIIS")
# ---------------------------------------------------------------------------

def _diis_run(f, V, o, mode, niter):
    t1, t2, t3 = R.mp2_guess(f, V, o)
    d = R.DIIS()
    out = []
    for _ in range(niter):
        j1, j2, j3 = t1, t2, t3
        t1, t2, t3, e, _ = R.iterate(f, V, t1, t2, t3, o, diis=d, diis_t3=mode)
        out.append((j1, j2, j3, t1, t2, t3, e))
    return out


def test_subspace_diis_over_all_virtuals_is_full_diis():
    """A subspace holding every virtual is the plain T3 DIIS, bit for bit."""
    o, v = 2, 4
    f, V = _tiny(o, v, 41)
    a = _diis_run(f, V, o, "full", 6)
    b = _diis_run(f, V, o, v, 6)
    for x, y in zip(a, b):
        assert x[6] == y[6]
        assert np.array_equal(x[5], y[5])


@pytest.mark.parametrize("mode", [2, "none"])
def test_t3_outside_the_diis_part_keeps_its_jacobi_step(mode):
    """Components of T3 that are not in the DIIS vectors equal the plain
    Jacobi update t + r/eps; the extrapolated ones (and T1, T2) do not."""
    o, v = 2, 4
    f, V = _tiny(o, v, 42)
    d1, d2, d3 = R.denominators(f, o)
    sub = 0 if mode == "none" else mode
    for j1, j2, j3, t1, t2, t3, _ in _diis_run(f, V, o, mode, 5)[2:]:
        r1, r2, r3 = R.residuals(f, V, j1, j2, j3, o)
        jac = j3 + R.postprocess_r3(r3) / d3
        outside = np.ones(t3.shape, bool)
        outside[:, :, :, :sub, :sub, :sub] = False
        assert np.array_equal(t3[outside], jac[outside])
        if sub:
            assert not np.allclose(t3[~outside], jac[~outside], rtol=0, atol=1e-14)
        assert not np.allclose(t1, j1 + r1 / d1, rtol=0, atol=1e-14)


def test_subspace_diis_converges_to_the_same_energy():
    """The accelerator does not move the fixed point: DIIS on a T3 subspace
    and on the whole T3 converge to the same RCCSDT energy."""
    o, v = 2, 4
    s = ci.make_system(o, v, 2 * (o + v), 43, sigma=0.1)  # a system plain Jacobi steps converge on
    f, V = s["f"], R.eri_phys_from_B(s["B"])
    ef, *_, itf, cf = R.solve(f, V, o, tol=1e-11, max_iter=300)
    es, *_, its, cs = R.solve(f, V, o, tol=1e-11, max_iter=300, diis_t3=2)
    en, *_, itn, cn = R.solve(f, V, o, tol=1e-11, max_iter=300, diis_t3="none")
    assert cf and cs and cn
    assert abs(ef - es) < 1e-12 and abs(ef - en) < 1e-12
