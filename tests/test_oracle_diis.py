"""CPU pins of the oracle's DIIS extrapolation (Sec. "Distributed DIIS": the
overlap matrix B_mn of the stored error vectors, the bordered linear system
for the coefficients, the extrapolated amplitudes).

What fixes the extrapolation independently of the oracle's own code:
* optimality: the coefficients minimise |sum_m c_m e_m| subject to
  sum_m c_m = 1.  Eliminating the constraint (c_M = 1 - sum_{m<M} c_m) turns
  this into an ordinary least-squares problem on the error VECTORS, solved
  here by numpy's lstsq (never forming B); the KKT conditions
  (B c)_m = lambda for every m are checked too;
* two vectors: c_1 = e_2.(e_2 - e_1) / |e_1 - e_2|^2, c_2 = 1 - c_1;
* Anderson / GMRES equivalence: on a linear fixed-point map x -> A x + b in
  dimension d, DIIS with a history of more than d vectors returns the exact
  fixed point from the (d+1)-th extrapolation on (d+1 error vectors in R^d
  have a combination that vanishes with coefficients summing to one);
* what is extrapolated: the Jacobi-updated vectors (reading c5), checked by
  feeding one-hot vectors so the output IS the coefficient vector, and by
  recording what the RCCSDT iteration passes in.
Planted mistakes (B from the vectors instead of the errors; extrapolating the
pre-step vectors) fail these pins.
"""

import numpy as np
import pytest

import cct_inputs as ci
from oracle import rccsdt as R


def lstsq_coefficients(errs):
    """argmin |sum c_m e_m| subject to sum c_m = 1, from the vectors."""
    E = np.stack(errs, axis=1)  # columns e_m
    M = E.shape[1]
    A = E[:, :-1] - E[:, -1:]  # e_m - e_M, m < M
    y, *_ = np.linalg.lstsq(A, -E[:, -1], rcond=None)
    return np.concatenate([y, [1.0 - y.sum()]])


def coefficients(diis_cls, errs, **kw):
    """Feed one-hot Jacobi vectors with the given errors; the extrapolated
    vector of the last update is then the coefficient vector itself."""
    M = len(errs)
    d = diis_cls(space=max(M, 2), start=2, **kw)
    out = None
    for m, e in enumerate(errs):
        vec = np.zeros(M)
        vec[m] = 1.0
        out = d.update(vec, e)
    return out


class FromVectors(R.DIIS):
    """Planted mistake: B built from the stored vectors instead of the errors."""

    def update(self, vec_new, err):
        return super().update(vec_new, vec_new.copy())


def test_two_vector_closed_form():
    rng = np.random.default_rng(1)
    e1, e2 = rng.normal(size=7), rng.normal(size=7)
    c = coefficients(R.DIIS, [e1, e2])
    c1 = e2 @ (e2 - e1) / ((e1 - e2) @ (e1 - e2))
    assert np.allclose(c, [c1, 1.0 - c1], rtol=0, atol=1e-13)


@pytest.mark.parametrize("M,n", [(3, 10), (5, 40), (8, 200)])
def test_coefficients_minimise_the_combined_error(M, n):
    rng = np.random.default_rng(M * 100 + n)
    errs = [rng.normal(size=n) * (0.5 ** k) for k in range(M)]
    c = coefficients(R.DIIS, errs)
    ref = lstsq_coefficients(errs)
    assert abs(c.sum() - 1.0) < 1e-13
    assert np.allclose(c, ref, rtol=0, atol=1e-10)
    # KKT: the gradient of |sum c e|^2 is the same for every coefficient
    E = np.stack(errs, axis=1)
    g = E.T @ (E @ c)
    assert np.ptp(g) < 1e-10 * max(1.0, np.abs(g).max())
    # the planted mistake gives other coefficients
    assert not np.allclose(coefficients(FromVectors, errs), ref, rtol=0, atol=1e-6)


@pytest.mark.parametrize("d", [3, 6, 10])
def test_linear_fixed_point_is_exact_after_d_plus_one_steps(d):
    """x <- A x + b: with history > d the (d+1)-th DIIS extrapolation of the
    Jacobi (here: plain map) steps is the exact fixed point."""
    rng = np.random.default_rng(7 + d)
    Q, _ = np.linalg.qr(rng.normal(size=(d, d)))
    A = Q @ np.diag(rng.uniform(-0.8, 0.8, d)) @ Q.T + 0.05 * rng.normal(size=(d, d))
    b = rng.normal(size=d)
    xstar = np.linalg.solve(np.eye(d) - A, b)

    def run(diis):
        x = np.zeros(d)
        outs = []
        for _ in range(d + 1):
            xj = A @ x + b
            x = diis.update(xj, xj - x)
            outs.append(x)
        return outs

    outs = run(R.DIIS(space=d + 2, start=2))
    err = np.abs(outs[d] - xstar).max() / np.abs(xstar).max()
    assert err < 1e-12, err
    # not merely converging: the plain map is far from the fixed point after d+1 steps
    x = np.zeros(d)
    for _ in range(d + 1):
        x = A @ x + b
    assert np.abs(x - xstar).max() / np.abs(xstar).max() > 1e-6

    class OldVectors(R.DIIS):
        """Planted mistake: extrapolate the pre-step vectors x_old = x_J - e."""

        def update(self, vec_new, err):
            return super().update(vec_new - err, err)

    bad = run(OldVectors(space=d + 2, start=2))
    assert np.abs(bad[d] - xstar).max() / np.abs(xstar).max() > 1e-8


def test_singular_system_drops_the_oldest_vector_for_good():
    """Two equal error vectors make the bordered system singular: the oldest
    vector leaves the history permanently (later solves do not see it)."""
    rng = np.random.default_rng(3)
    e = rng.normal(size=5)
    d = R.DIIS(space=8, start=2)
    d.update(np.array([1.0, 0.0, 0.0]), e)
    out = d.update(np.array([0.0, 1.0, 0.0]), e.copy())
    assert np.array_equal(out, [0.0, 1.0, 0.0]) and len(d.vecs) == 1
    e3 = rng.normal(size=5)
    out = d.update(np.array([0.0, 0.0, 1.0]), e3)
    c = lstsq_coefficients([e, e3])
    assert np.allclose(out, [0.0, c[0], c[1]], rtol=0, atol=1e-13)


def test_rccsdt_iteration_extrapolates_the_jacobi_vectors():
    """The iteration hands DIIS the Jacobi-updated amplitudes t + r/eps and the
    error (t + r/eps) - t, and returns DIIS's output as the new amplitudes."""
    o, v = 2, 3
    s = ci.make_system(o, v, 2 * (o + v), 5, sigma=0.1)
    f, V = s["f"], R.eri_phys_from_B(s["B"])
    t1, t2, t3 = R.mp2_guess(f, V, o)

    class Recorder(R.DIIS):
        def __init__(self):
            super().__init__()
            self.seen = []

        def update(self, vec_new, err):
            self.seen.append((vec_new.copy(), err.copy()))
            out = super().update(vec_new, err)
            self.seen[-1] += (out.copy(),)
            return out

    d = Recorder()
    for _ in range(3):
        r1, r2, r3 = R.residuals(f, V, t1, t2, t3, o)
        d1, d2, d3 = R.denominators(f, o)
        jac = R.pack_vec(t1 + r1 / d1, t2 + r2 / d2, t3 + R.postprocess_r3(r3) / d3)
        old = R.pack_vec(t1, t2, t3)
        t1, t2, t3, e, _ = R.iterate(f, V, t1, t2, t3, o, diis=d)
        vec, err, out = d.seen[-1]
        assert np.array_equal(vec, jac)
        assert np.array_equal(err, jac - old)
        assert np.array_equal(R.pack_vec(t1, t2, t3), out)
