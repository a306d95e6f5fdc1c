"""Equation-free brute force in determinant space (test oracle only).

* Full CI in a fixed electron-number / S_z sector.
* Spin-orbital projective coupled cluster: for amplitudes t_mu the residual is
  r_mu = <Phi_mu| exp(-T) H exp(T) |Phi_0> and the energy is
  <Phi_0| exp(-T) H exp(T) |Phi_0> (Appendix A, "Coupled-cluster theory"),
  evaluated with explicit operator matrices; T is nilpotent so both
  exponential series are finite.  |Phi_mu> = tau_mu |Phi_0>, where
  tau_mu = a+_{A1}...a+_{An} a_{In}...a_{I1} is the operator that multiplies
  t_mu in T, so that <Phi_mu|tau_mu|Phi_0> = 1.
* The spin-free <-> spin-orbital amplitude maps of the spin-free formalism:
  M (spin-free t -> antisymmetric spin-orbital t, via the antisymmetrisers over
  virtual labels restricted to spin-matched columns) and L (the closed-shell
  reconstruction of the spin-free T3 from the spin-orbital T3 given at the end
  of the UCCSDT appendix).

Spin orbital P = 2p + s for spatial orbital p and spin s (0 = alpha, 1 = beta).
Hamiltonian H = sum h_PQ a+_P a_Q + 1/2 sum <PQ|RS> a+_P a+_Q a_S a_R with
<PQ|RS> = (pr|qs) delta(s_P,s_R) delta(s_Q,s_S) and h = f - sum_i (2J_i - K_i)
over the doubly occupied reference orbitals (Appendix A, "Hamiltonian").
"""

from __future__ import annotations

import itertools
from math import factorial

import numpy as np
import scipy.sparse as sp


# ----------------------------------------------------------------------------
# Determinant spaces and elementary operators on bit strings
# ----------------------------------------------------------------------------

def _dets(nso, nel, sz2=None):
    out = []
    for occ in itertools.combinations(range(nso), nel):
        if sz2 is not None:
            na = sum(1 for p in occ if p % 2 == 0)
            if na - (nel - na) != sz2:
                continue
        d = 0
        for p in occ:
            d |= 1 << p
        out.append(d)
    return np.array(sorted(out), dtype=np.int64)


def _apply_ops(dets, ops):
    """Apply a product of elementary operators to an array of determinants.
    ``ops`` lists (kind, orbital) in the order they act (rightmost first);
    kind 0 = annihilate, 1 = create.  Returns (new dets, sign, valid)."""
    cur = dets.copy()
    sign = np.ones(dets.shape, dtype=np.int64)
    valid = np.ones(dets.shape, dtype=bool)
    for kind, p in ops:
        bit = np.int64(1) << np.int64(p)
        occ = (cur & bit) != 0
        valid &= occ if kind == 0 else ~occ
        below = cur & (bit - np.int64(1))
        par = np.bitwise_count(below) & 1
        sign *= np.where(par == 1, -1, 1)
        cur = cur ^ bit
    return cur, sign, valid


def _lookup(space, dets):
    idx = np.searchsorted(space, dets)
    idx = np.clip(idx, 0, len(space) - 1)
    found = space[idx] == dets
    return idx, found


class SpinOrbitalSystem:
    """Spin-orbital Hamiltonian of a closed-shell spatial problem and operator
    machinery in one N-electron S_z sector."""

    def __init__(self, f, V, o, nel=None, ref_occ=None):
        n = f.shape[0]
        self.n, self.o = n, o
        self.nso = 2 * n
        # h = f - sum_i (2 v^{pi}_{qi} - v^{pi}_{iq}) over doubly occupied reference orbitals
        h = f - (2.0 * np.einsum("piqi->pq", V[:, :o, :, :o]) - np.einsum("piiq->pq", V[:, :o, :o, :]))
        self.h_spatial = h
        if ref_occ is None:
            ref_occ = list(range(2 * o)) if nel is None else list(range(nel))
        self.ref_occ = sorted(ref_occ)
        self.nel = len(self.ref_occ)
        nso = self.nso
        spin = np.arange(nso) % 2
        sp_ = np.arange(nso) // 2
        hso = h[sp_[:, None], sp_[None, :]] * (spin[:, None] == spin[None, :])
        self.hso = hso
        # Vso[P,Q,R,S] = <PQ|RS> = V[p,q,r,s] delta(sP,sR) delta(sQ,sS)
        Vso = V[np.ix_(sp_, sp_, sp_, sp_)].copy()
        Vso *= (spin[:, None, None, None] == spin[None, None, :, None])
        Vso *= (spin[None, :, None, None] == spin[None, None, None, :])
        self.Vso = Vso
        na = sum(1 for p in self.ref_occ if p % 2 == 0)
        self.sz2 = na - (self.nel - na)
        self.space = _dets(nso, self.nel, self.sz2)
        self.space1 = _dets(nso, self.nel - 1)
        self.space2 = _dets(nso, self.nel - 2) if self.nel >= 2 else None
        ref = 0
        for p in self.ref_occ:
            ref |= 1 << p
        self.ref = ref
        self.ref_index = int(np.searchsorted(self.space, ref))
        self._build_h_maps()

    # --- Hamiltonian -------------------------------------------------------
    def _build_h_maps(self):
        nso = self.nso
        D = self.space
        self.one = []
        for P in range(nso):
            nd, sg, ok = _apply_ops(D, [(0, P)])
            idx, found = _lookup(self.space1, nd)
            ok &= found
            self.one.append((np.nonzero(ok)[0], idx[ok], sg[ok]))
        self.two = []
        self.pairs = []
        if self.space2 is None:
            return
        for P in range(nso):
            for Q in range(nso):
                if P == Q:
                    continue
                # G_PQ = a_Q a_P (a_P acts first)
                nd, sg, ok = _apply_ops(D, [(0, P), (0, Q)])
                idx, found = _lookup(self.space2, nd)
                ok &= found
                self.pairs.append((P, Q))
                self.two.append((np.nonzero(ok)[0], idx[ok], sg[ok]))
        npair = len(self.pairs)
        Vm = np.empty((npair, npair))
        for a, (P, Q) in enumerate(self.pairs):
            for b, (R, S) in enumerate(self.pairs):
                Vm[a, b] = self.Vso[P, Q, R, S]
        self.Vpair = Vm

    def apply_h(self, psi):
        """H psi for psi of shape (dim,) or (dim, m)."""
        vec = psi.ndim == 1
        X = psi[:, None] if vec else psi
        m = X.shape[1]
        out = np.zeros_like(X)
        # one-body: sum_PQ h_PQ a+_P a_Q
        Y1 = np.zeros((self.nso, len(self.space1), m))
        for Q, (src, tgt, sg) in enumerate(self.one):
            np.add.at(Y1[Q], tgt, sg[:, None] * X[src])
        Z1 = np.einsum("PQ,Qtm->Ptm", self.hso, Y1)
        for P, (src, tgt, sg) in enumerate(self.one):
            np.add.at(out, src, sg[:, None] * Z1[P, tgt])
        # two-body: 1/2 sum <PQ|RS> (a_Q a_P)^T (a_S a_R)
        if self.space2 is not None:
            npair = len(self.pairs)
            Y2 = np.zeros((npair, len(self.space2), m))
            for a, (src, tgt, sg) in enumerate(self.two):
                np.add.at(Y2[a], tgt, sg[:, None] * X[src])
            Z2 = np.einsum("ab,btm->atm", self.Vpair, Y2)
            for a, (src, tgt, sg) in enumerate(self.two):
                np.add.at(out, src, 0.5 * sg[:, None] * Z2[a, tgt])
        return out[:, 0] if vec else out

    def hf_energy(self):
        e0 = np.zeros(len(self.space))
        e0[self.ref_index] = 1.0
        return float(self.apply_h(e0)[self.ref_index])

    def fci(self, chunk=128):
        """Lowest eigenvalue of H in the sector (dense diagonalisation)."""
        dim = len(self.space)
        H = np.empty((dim, dim))
        for c0 in range(0, dim, chunk):
            c1 = min(dim, c0 + chunk)
            E = np.zeros((dim, c1 - c0))
            E[np.arange(c0, c1), np.arange(c1 - c0)] = 1.0
            H[:, c0:c1] = self.apply_h(E)
        H = 0.5 * (H + H.T)
        w = np.linalg.eigvalsh(H)
        return float(w[0])

    # --- excitations and cluster operator ----------------------------------
    def excitations(self, max_rank):
        """All S_z-conserving excitations (I sorted, A sorted) of rank 1..max_rank
        out of the reference."""
        occ = self.ref_occ
        vir = [p for p in range(self.nso) if p not in occ]
        out = []
        for rank in range(1, max_rank + 1):
            for I in itertools.combinations(occ, rank):
                for A in itertools.combinations(vir, rank):
                    if sum(p % 2 for p in I) != sum(p % 2 for p in A):
                        continue
                    out.append((I, A))
        return out

    def _tau_ops(self, I, A):
        # tau = a+_{A1} ... a+_{An} a_{In} ... a_{I1}: a_{I1} acts first
        ops = [(0, p) for p in I]
        ops += [(1, p) for p in reversed(A)]
        return ops

    def prepare(self, excs):
        """Precompute the matrix entries of every tau_mu in the sector and the
        (index, sign) of tau_mu |Phi_0>."""
        self.excs = list(excs)
        rows, cols, signs, owner = [], [], [], []
        ref_pos = []
        D = self.space
        for mu, (I, A) in enumerate(self.excs):
            nd, sg, ok = _apply_ops(D, self._tau_ops(I, A))
            idx, found = _lookup(D, nd)
            ok &= found
            src = np.nonzero(ok)[0]
            rows.append(idx[ok])
            cols.append(src)
            signs.append(sg[ok])
            owner.append(np.full(len(src), mu))
            r_nd, r_sg, r_ok = _apply_ops(np.array([self.ref], dtype=np.int64), self._tau_ops(I, A))
            assert r_ok[0]
            ref_pos.append((int(np.searchsorted(D, r_nd[0])), int(r_sg[0])))
        self._rows = np.concatenate(rows)
        self._cols = np.concatenate(cols)
        self._signs = np.concatenate(signs).astype(float)
        self._owner = np.concatenate(owner)
        self._ref_pos = ref_pos

    def t_matrix(self, t):
        dim = len(self.space)
        data = self._signs * np.asarray(t)[self._owner]
        return sp.csr_matrix((data, (self._rows, self._cols)), shape=(dim, dim))

    def _exp_apply(self, T, psi, sgn):
        out = psi.copy()
        term = psi.copy()
        for k in range(1, self.nel + 2):
            term = (T @ term) * (sgn / k)
            if not np.any(term):
                break
            out += term
        return out

    def cc_residual(self, t):
        """(E_total, r) with r_mu = <Phi_mu| exp(-T) H exp(T) |Phi_0>."""
        T = self.t_matrix(t)
        psi = np.zeros(len(self.space))
        psi[self.ref_index] = 1.0
        psi = self._exp_apply(T, psi, 1.0)
        hpsi = self.apply_h(psi)
        hbar = self._exp_apply(T, hpsi, -1.0)
        r = np.array([sg * hbar[pos] for (pos, sg) in self._ref_pos])
        return float(hbar[self.ref_index]), r

    def amplitudes_from_ci(self, c):
        """Cluster amplitudes of a full-rank expansion: exp(T)|Phi_0> = c / c_0,
        so T|Phi_0> = log(1 + C)|Phi_0> with C built from the excited
        coefficients (excitation operators commute)."""
        c = c / c[self.ref_index]
        cvec = np.array([sg * c[pos] for (pos, sg) in self._ref_pos])
        C = self.t_matrix(cvec)
        phi = np.zeros(len(self.space))
        phi[self.ref_index] = 1.0
        out = np.zeros_like(phi)
        term = phi.copy()
        for k in range(1, self.nel + 2):
            term = C @ term
            if not np.any(term):
                break
            out += ((-1.0) ** (k + 1) / k) * term
        return np.array([sg * out[pos] for (pos, sg) in self._ref_pos])

    def q_correction(self, tso, eps):
        """Perturbative quadruples energy from spin-orbital T2, T3 (entries of
        ``tso`` on the excitations passed to ``prepare``, which must include
        rank 4; other ranks are ignored) and spatial orbital energies ``eps``:

          E = sum_Q <Q|H_N (T2 + T3)|0> <Q|H_N T3 + 1/2 (H_N T2^2)_C|0> / D_Q

        over the unique quadruply excited determinants Q, with
        H_N = H - <0|H|0> and D_Q = sum eps_occ - sum eps_vir.  The connected
        part of H_N T2^2 / 2 on quadruples is the whole term minus
        (H_N T2)_C T2, where (H_N T2)_C is the doubles projection of H_N T2|0>
        read back as an excitation operator (its only non-vanishing rank on
        quadruples; excitation operators commute).  Canonical reference: the
        Fock matrix of |Phi_0> is diagonal, so H_N has no pure one-body
        excitation part."""
        rank = np.array([len(I) for I, _ in self.excs])
        tso = np.asarray(tso, dtype=float)
        T2 = self.t_matrix(np.where(rank == 2, tso, 0.0))
        T3 = self.t_matrix(np.where(rank == 3, tso, 0.0))
        e_ref = self.hf_energy()
        phi = np.zeros(len(self.space))
        phi[self.ref_index] = 1.0

        def hn(x):
            return self.apply_h(x) - e_ref * x

        def proj(x):
            return np.array([sg * x[pos] for (pos, sg) in self._ref_pos])

        a2 = T2 @ phi
        a3 = T3 @ phi
        x2 = np.where(rank == 2, proj(hn(a2)), 0.0)
        left = proj(hn(a2 + a3))
        right = proj(hn(a3) + 0.5 * hn(T2 @ a2) - self.t_matrix(x2) @ a2)
        e = 0.0
        for mu, (I, A) in enumerate(self.excs):
            if len(I) != 4:
                continue
            d = sum(eps[P // 2] for P in I) - sum(eps[P // 2] for P in A)
            e += left[mu] * right[mu] / d
        return float(e)

    def fci_vector(self):
        dim = len(self.space)
        H = np.empty((dim, dim))
        for c0 in range(0, dim, 128):
            c1 = min(dim, c0 + 128)
            E = np.zeros((dim, c1 - c0))
            E[np.arange(c0, c1), np.arange(c1 - c0)] = 1.0
            H[:, c0:c1] = self.apply_h(E)
        w, U = np.linalg.eigh(0.5 * (H + H.T))
        return float(w[0]), U[:, 0]


# ----------------------------------------------------------------------------
# Spin-free <-> spin-orbital maps
# ----------------------------------------------------------------------------

def _perm_sign(p):
    p = list(p)
    s = 1
    for a in range(len(p)):
        for b in range(a + 1, len(p)):
            if p[a] > p[b]:
                s = -s
    return s


def spinfree_to_spinorb(excs, o, t1, t2, t3, t4=None):
    """Map M: t_{I1..In}^{A1..An} = sum_pi sgn(pi) prod_k delta(s(I_k), s(A_pi(k)))
    tchk_{i1..in}^{a_pi(1)..a_pi(n)}, i.e. antisymmetrisation over virtual labels
    restricted to spin-matched columns (t_{ij kbar}^{ab cbar} = A^{ab} t,
    t_{ijk}^{abc} = A^{abc} t, t_{i jbar}^{a bbar} = t_ij^ab); quadruples (t4)
    alike when given."""
    amps = {1: t1, 2: t2, 3: t3}
    if t4 is not None:
        amps[4] = t4
    out = np.zeros(len(excs))
    for mu, (I, A) in enumerate(excs):
        n = len(I)
        tt = amps.get(n)
        if tt is None:
            continue
        occ = [P // 2 for P in I]
        vir = [P // 2 - o for P in A]
        val = 0.0
        for pi in itertools.permutations(range(n)):
            if any(I[k] % 2 != A[pi[k]] % 2 for k in range(n)):
                continue
            val += _perm_sign(pi) * tt[tuple(occ) + tuple(vir[pi[k]] for k in range(n))]
        out[mu] = val
    return out


class SpinOrbAccessor:
    """Antisymmetric access r(I-list, A-list) for arbitrary index orders."""

    def __init__(self, excs, vals):
        self.tab = {(tuple(I), tuple(A)): x for (I, A), x in zip(excs, vals)}

    def __call__(self, I, A):
        if len(set(I)) < len(I) or len(set(A)) < len(A):
            return 0.0
        oi = sorted(range(len(I)), key=lambda s: I[s])
        oa = sorted(range(len(A)), key=lambda s: A[s])
        key = (tuple(I[s] for s in oi), tuple(A[s] for s in oa))
        return _perm_sign(oi) * _perm_sign(oa) * self.tab.get(key, 0.0)


def spinorb_to_spinfree(excs, vals, o, v):
    """Spin-free singles/doubles from the spin-orbital ones, r_i^a = r_{i alpha}^{a alpha},
    r_ij^ab = r_{i alpha j beta}^{a alpha b beta}, and triples by the map L:
    t_ijk^abc = -1/6 t_{ijk}^{abc}(alpha^3)
                + 1/3 (t_{ij kbar}^{ab cbar} + t_{ik jbar}^{ac bbar} + t_{jk ibar}^{bc abar})."""
    acc = SpinOrbAccessor(excs, vals)
    al = lambda p: 2 * p
    be = lambda p: 2 * p + 1
    V = lambda a: o + a
    r1 = np.zeros((o, v))
    r2 = np.zeros((o, o, v, v))
    r3 = np.zeros((o, o, o, v, v, v))
    for i in range(o):
        for a in range(v):
            r1[i, a] = acc([al(i)], [al(V(a))])
    for i, j in itertools.product(range(o), repeat=2):
        for a, b in itertools.product(range(v), repeat=2):
            r2[i, j, a, b] = acc([al(i), be(j)], [al(V(a)), be(V(b))])
    for i, j, k in itertools.product(range(o), repeat=3):
        for a, b, c in itertools.product(range(v), repeat=3):
            x = -acc([al(i), al(j), al(k)], [al(V(a)), al(V(b)), al(V(c))]) / 6.0
            x += (acc([al(i), al(j), be(k)], [al(V(a)), al(V(b)), be(V(c))])
                  + acc([al(i), al(k), be(j)], [al(V(a)), al(V(c)), be(V(b))])
                  + acc([al(j), al(k), be(i)], [al(V(b)), al(V(c)), be(V(a))])) / 3.0
            r3[i, j, k, a, b, c] = x
    return r1, r2, r3


def solve_cc(sysm: SpinOrbitalSystem, max_rank, tol=1e-11, max_iter=200):
    """Projective spin-orbital CC by Newton iterations with a finite-difference
    Jacobian (tiny problems only).  Returns (E_corr, t, converged)."""
    excs = sysm.excitations(max_rank)
    sysm.prepare(excs)
    ehf = sysm.hf_energy()
    t = np.zeros(len(excs))
    for it in range(max_iter):
        e, r = sysm.cc_residual(t)
        if np.linalg.norm(r) < tol:
            return e - ehf, t, True
        J = np.empty((len(r), len(t)))
        h = 1e-6
        for m in range(len(t)):
            tp = t.copy()
            tp[m] += h
            J[:, m] = (sysm.cc_residual(tp)[1] - r) / h
        t = t - np.linalg.solve(J, r)
    e, r = sysm.cc_residual(t)
    return e - ehf, t, False


def nfact(n):
    return factorial(n)
