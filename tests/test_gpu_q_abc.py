"""GPU: E_(Q) in the virtual-tuple order (cct_energy_q_abc, Sec. "ABC-based
algorithm", Eq. ener-pt-q-abc with the intermediates of Eq. q_w_alter)
against the (Q) oracle.

* small systems, every task: the total against the oracle's full-tensor
  E_(Q), each task against the oracle's one-tuple evaluation in the
  virtual-tuple order summed over the task's tuples a <= b <= c <= d, and
  every tuple's share one by one; tuples with three equal labels give
  exactly 0.  Shapes cover odd v (scalar operand loads), ragged last tiles,
  a single tile (every slot in one tile), tiles of one label and a task
  subset;
* the occupied-tuple GPU path (cct_energy_q) on the same amplitudes, at
  sizes the full-tensor oracle cannot hold;
* o=20, v=180 (the benchmark's workload, weak-coupling integrals, T2/T3
  after one iteration from MP2), block 4 as the benchmark runs it: the
  shares of sampled tuples of two tasks against the oracle's one-tuple
  evaluation, whose T3 slices are gathered from the device's packed T3
  element by element and whose integrals are built from the factors.
"""

import itertools
import sys

import numpy as np
import pytest

import cct_inputs as ci
from oracle import rccsdt as R, rccsdt_q as Q
from paper_2607_00981_amd import binding

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _random_case(o, v, seed):
    s = ci.make_system(o, v, 2 * (o + v), seed, sigma=0.1)
    _, t2, t3 = ci.random_amplitudes(o, v, seed + 1, 0.02, 0.05, 0.05)
    t3 = R.orthogonalize_r3(R.purify_r3(t3))
    return s, t2, t3


def _tile_quads(v, nb):
    nt = (v + nb - 1) // nb
    return [q for q in itertools.combinations_with_replacement(range(nt), 4)]


def _box(q, v, nb):
    """Tuples of a task's box in row-major order over the four tiles."""
    rng = [range(t * nb, min((t + 1) * nb, v)) for t in q]
    return list(itertools.product(*rng))


def _counted(tau):
    a, b, c, d = tau
    return a <= b <= c <= d and not (a == b == c) and not (b == c == d)


@pytest.mark.parametrize("o,v,nb,seed", [(2, 5, 2, 1), (3, 7, 3, 2), (3, 8, 4, 3), (2, 6, 6, 4), (2, 9, 4, 5),
                                         (3, 4, 1, 6)])
def test_q_abc_matches_oracle(o, v, nb, seed):
    say(f"[q_abc] o={o} v={v} block={nb} seed={seed}")
    s, t2, t3 = _random_case(o, v, seed)
    f, B = s["f"], s["B"]
    V = R.eri_phys_from_B(B)
    e_ref = Q.energy_q(f, V, t2, t3, o)
    quads = _tile_quads(v, nb)
    assert binding.q_abc_task_count(v, nb) == len(quads)
    with binding.Engine(o, v, B.shape[0]) as eng:
        eng.set_fock(f)
        eng.set_eri_df(B)
        eng.set_amplitudes(np.zeros((o, v)), t2, R.pack_t3(t3))
        res = eng.energy_q_abc(nb, tuples=True)
    say(f"  gpu {res['e_q']:.15e} oracle {e_ref:.15e} diff {res['e_q'] - e_ref:.2e}")
    assert abs(e_ref) > 1e-7
    assert abs(res["e_q"] - e_ref) <= 1e-13 + 1e-11 * abs(e_ref)
    scale = 0.0
    tuple_ref = {}
    for tau in itertools.combinations_with_replacement(range(v), 4):
        tuple_ref[tau] = Q.virtual_task_energy(f, V, t2, t3, o, tau) if _counted(tau) else 0.0
        scale = max(scale, abs(tuple_ref[tau]))
    for k, q in enumerate(quads):
        box = _box(q, v, nb)
        got = res["e_tuples"][k]
        ref_task = 0.0
        for m, tau in enumerate(box):
            ref = tuple_ref[tau] if _counted(tau) else 0.0
            ref_task += ref
            if not _counted(tau):
                assert got[m] == 0.0, (q, tau)
            else:
                assert abs(got[m] - ref) <= 1e-13 * scale + 1e-11 * abs(ref), (q, tau, got[m], ref)
        assert np.all(got[len(box):] == 0.0)
        assert abs(res["e_tasks"][k] - ref_task) <= 1e-12 * scale, (q, res["e_tasks"][k], ref_task)


def test_q_abc_task_subset_and_errors():
    o, v, nb = 3, 7, 2
    say(f"[q_abc] task subset o={o} v={v} block={nb}")
    s, t2, t3 = _random_case(o, v, 12)
    with binding.Engine(o, v, s["B"].shape[0]) as eng:
        eng.set_fock(s["f"])
        eng.set_eri_df(s["B"])
        eng.set_amplitudes(np.zeros((o, v)), t2, R.pack_t3(t3))
        full = eng.energy_q_abc(nb)
        pick = [7, 0, 33, 7]
        part = eng.energy_q_abc(nb, tasks=pick)
        assert np.array_equal(part["e_tasks"], full["e_tasks"][pick])
        assert part["e_q"] == sum(float(x) for x in full["e_tasks"][pick])
        empty = eng.energy_q_abc(nb, tasks=[])
        assert empty["e_q"] == 0.0
        for bad in (0, 17, v + 1):
            with pytest.raises(binding.CCTError) as e:
                eng.energy_q_abc(bad)
            assert e.value.code == binding.CCT_EINVAL
        with pytest.raises(binding.CCTError) as e:
            eng.energy_q_abc(nb, tasks=[binding.q_abc_task_count(v, nb)])
        assert e.value.code == binding.CCT_EINVAL


@pytest.mark.parametrize("o,v,nb,seed", [(5, 23, 4, 21), (6, 24, 8, 22), (4, 30, 16, 23)])
def test_q_abc_equals_occupied_order(o, v, nb, seed):
    say(f"[q_abc] vs occupied-tuple path o={o} v={v} block={nb}")
    s, t2, t3 = _random_case(o, v, seed)
    with binding.Engine(o, v, s["B"].shape[0]) as eng:
        eng.set_fock(s["f"])
        eng.set_eri_df(s["B"])
        eng.set_amplitudes(np.zeros((o, v)), t2, R.pack_t3(t3))
        e_ijk = eng.energy_q()
        e_abc = eng.energy_q_abc(nb)["e_q"]
    say(f"  abc {e_abc:.15e} ijk {e_ijk:.15e} diff {e_abc - e_ijk:.2e}")
    assert abs(e_ijk) > 1e-7
    assert abs(e_abc - e_ijk) <= 1e-11 * abs(e_ijk)


class _LazyV:
    """v^{pq}_{rs} = sum_P B[P,p,r] B[P,q,s] for the index sets requested."""

    def __init__(self, B):
        self.B = B

    def __getitem__(self, key):
        n = self.B.shape[1]
        ix = [np.arange(n)[k] if isinstance(k, slice) else np.array([k]) for k in key]
        L = self.B[:, ix[0]][:, :, ix[2]]
        Rr = self.B[:, ix[1]][:, :, ix[3]]
        out = np.einsum("Ppr,Pqs->pqrs", L, Rr, optimize=True)
        return out[tuple(0 if not isinstance(k, slice) else slice(None) for k in key)]


class _LazyT3:
    """Full-tensor indexing t3[i, j, k, a, b, c] served from the device's
    packed T3 (block sort(i, j, k), virtual axes permuted alike)."""

    def __init__(self, eng, o, v):
        self.eng, self.o, self.v = eng, o, v
        tri = np.full((o, o, o), -1, dtype=np.int64)
        for i in range(o):
            for j in range(i, o):
                for k in range(j, o):
                    tri[i, j, k] = binding.packed_index(o, i, j, k)
        self.tri = tri
        self.cache = {}

    def __getitem__(self, key):
        ck = tuple((k.start, k.stop, k.step) if isinstance(k, slice) else int(k) for k in key)
        if ck in self.cache:
            return self.cache[ck]
        o, v = self.o, self.v
        ax = [np.arange(o if d < 3 else v)[k] if isinstance(k, slice) else np.array([k]) for d, k in enumerate(key)]
        g = np.meshgrid(*ax, indexing="ij")
        occ = np.stack([g[0].ravel(), g[1].ravel(), g[2].ravel()])
        vir = np.stack([g[3].ravel(), g[4].ravel(), g[5].ravel()])
        order = np.argsort(occ, axis=0, kind="stable")
        so = np.take_along_axis(occ, order, 0)
        sv = np.take_along_axis(vir, order, 0)
        t = self.tri[so[0], so[1], so[2]]
        flat = ((t * v + sv[0]) * v + sv[1]) * v + sv[2]
        vals = self.eng.gather_t3(flat).reshape(g[0].shape)
        out = vals[tuple(0 if not isinstance(k, slice) else slice(None) for k in key)]
        self.cache[ck] = out
        return out


def test_q_abc_o20v180_sampled_tuples_match_oracle():
    s = ci.make_named("o20v180-weak")
    o, v, naux, nb = s["o"], s["v"], s["naux"], 4
    say(f"[q_abc] o={o} v={v} block={nb}: one iteration from MP2, then two tasks")
    quads = _tile_quads(v, nb)
    index = {q: k for k, q in enumerate(quads)}
    picks = [(0, 5, 17, 44), (3, 3, 10, 20)]
    with binding.Engine(o, v, naux, precision="bf16x3", opts={"diis_t3": "none"}) as eng:
        eng.set_fock(s["f"])
        eng.set_eri_df(s["B"])
        eng.init_mp2()
        eng.update()
        res = eng.energy_q_abc(nb, tasks=[index[q] for q in picks], tuples=True)
        say(f"  tasks {res['e_tasks']} stats {res['stats']}")
        _, t2, _ = eng.get_amplitudes(with_t3=False)
        t3 = _LazyT3(eng, o, v)
        V = _LazyV(s["B"])
        checked = 0
        for k, q in enumerate(picks):
            box = _box(q, v, nb)
            got = res["e_tuples"][k]
            # sampled tuples: first, last, the first with four distinct labels and
            # the first with a repeated label (if the box has one)
            cand = [m for m, tau in enumerate(box) if _counted(tau)]
            rep = [m for m in cand if len(set(box[m])) < 4]
            dis = [m for m in cand if len(set(box[m])) == 4]
            sample = sorted(set([cand[0], cand[-1]] + rep[:1] + dis[:1]))
            for m in sample:
                tau = box[m]
                ref = Q.virtual_task_energy(s["f"], V, t2, t3, o, tau)
                say(f"  tuple {tau}: gpu {got[m]:.15e} oracle {ref:.15e}")
                assert abs(ref) > 0.0
                assert abs(got[m] - ref) <= 1e-12 * abs(ref) + 1e-18
                checked += 1
            assert all(got[m] == 0.0 for m, tau in enumerate(box) if not _counted(tau))
            assert abs(res["e_tasks"][k] - sum(float(x) for x in got)) <= 1e-12 * np.abs(got).sum()
        assert checked >= 5
