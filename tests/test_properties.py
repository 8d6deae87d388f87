"""Property sweeps (hypothesis) over the host-side argument rules of the C ABI
and over the FP64 oracle's mathematical invariants, at random small shapes.

The C ABI sweeps call only host entry points (workspace sizing, batch
creation, checkpoint checks), so they need no GPU.  The oracle sweeps check
facts that hold for any input:

* the sketch's singular values interlace with A's (sigma_i(Q Q^T A) <= sigma_i(A));
* a sketch as wide as min(m, n) gives the exact SVD (Alg. rqb with l = min(m, n));
* a matrix of exact rank r is reproduced once l >= r (Sec. 3, exact rank);
* the factors are orthonormal, sigma is sorted and non-negative, and the
  sign rule leaves the largest-magnitude entry of each v_i positive;
* the QR and LU normalisations of the power iterations span the same space
  (Alg. subspace_iter and Alg. normalized_iter agree in exact arithmetic);
* the column ID reproduces the chosen columns exactly (Z[:, J] = I, Sec. 6);
* soft thresholding is the proximal map of tau ||.||_1 (Sec. 5).
"""
import ctypes

import numpy as np
import pytest
from hypothesis import HealthCheck, assume, given, settings
from hypothesis import strategies as st

from oracle import learned as lrn
from oracle import philox
from oracle import rid as orid
from oracle import rrpca as orr
from oracle import rsvd as orc
from paper_1608_02148_amd import lib as L

FAST = settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.function_scoped_fixture])
SLOW = settings(max_examples=25, deadline=None, suppress_health_check=[HealthCheck.function_scoped_fixture])


@pytest.fixture(scope="module")
def lib():
    return L.load()


@pytest.fixture(scope="module")
def handle(lib):
    h = ctypes.c_void_p()
    assert lib.rsvd_create(ctypes.byref(h), None) == 0
    yield h
    lib.rsvd_destroy(h)


def _expected_status(dtype, m, n, k, p, q, sdist, precision, scheme, probes):
    """The argument rules the header states for rsvd_workspace_size."""
    if dtype not in (L.RSVD_F64, L.RSVD_F32, L.RSVD_BF16):
        return -2
    if m < 1 or n < 1 or k < 1 or k >= min(m, n) or p < 0 or q < 0:
        return -1
    if sdist not in (0, 1, 2):
        return -1
    if precision not in (0, 1) or (precision == 1 and dtype == L.RSVD_F64):
        return -2
    if probes < 0 or probes > 16 or scheme not in (0, 1):
        return -1
    l = min(k + p, min(m, n))
    if l > 256 or (scheme == 1 and l > 128):
        return -2
    return 0


@FAST
@given(dtype=st.sampled_from([0, 1, 2, 5]), m=st.integers(0, 300000), n=st.integers(0, 20000),
       k=st.integers(-2, 300), p=st.integers(-2, 60), q=st.integers(-1, 4), sdist=st.integers(-1, 3),
       precision=st.integers(0, 2), scheme=st.integers(0, 2), probes=st.integers(-1, 17))
def test_workspace_rules_and_size(lib, handle, dtype, m, n, k, p, q, sdist, precision, scheme, probes):
    prm = L.Params()
    lib.rsvd_default_params(ctypes.byref(prm))
    prm.p, prm.q, prm.sdist, prm.precision, prm.scheme, prm.probes = p, q, sdist, precision, scheme, probes
    out = ctypes.c_size_t(0)
    got = lib.rsvd_workspace_size(handle, dtype, m, n, k, ctypes.byref(prm), ctypes.byref(out))
    assert got == _expected_status(dtype, m, n, k, p, q, sdist, precision, scheme, probes)
    if got == 0:
        cs = {L.RSVD_F64: 8, L.RSVD_F32: 4, L.RSVD_BF16: 4}[dtype]
        l = min(k + p, min(m, n))
        # the workspace holds at least the two bases and Omega at width l
        assert out.value % 256 == 0 and out.value >= (m + 2 * n) * l * cs


@FAST
@given(shapes=st.lists(st.tuples(st.integers(8, 3000), st.integers(8, 3000), st.integers(1, 40)),
                       min_size=1, max_size=12))
def test_batch_creation_rules(lib, handle, shapes):
    """A batch is accepted exactly when every member passes the single-solve
    rules at the batch width limit, and its workspace covers each member's
    bases and Omega."""
    arr = (L.BatchDesc * len(shapes))()
    for b, (m, n, k) in enumerate(shapes):
        d = arr[b]
        d.A, d.lda, d.m, d.n, d.k, d.stream_id = 4096 * (b + 1), n, m, n, k, b
        d.U, d.ldu = 1 << 20, k
        d.S, d.V, d.ldv, d.info = 1 << 21, 1 << 22, k, None
        d.features, d.q, d.p = None, -1, -1
    prm = L.Params()
    lib.rsvd_default_params(ctypes.byref(prm))
    bh = ctypes.c_void_p()
    ws = ctypes.c_size_t(0)
    got = lib.rsvd_batch_create(handle, L.RSVD_F32, len(shapes), arr, ctypes.byref(prm), 0, ctypes.byref(bh),
                                ctypes.byref(ws))
    ok = all(1 <= k < min(m, n) and min(k + 10, min(m, n)) <= 128 for m, n, k in shapes)
    assert (got == 0) == ok and got in (0, -1, -2)
    if got == 0:
        need = max((m + 2 * n) * min(k + 10, min(m, n)) * 4 for m, n, k in shapes)
        assert ws.value >= need and ws.value % 256 == 0
        lib.rsvd_batch_destroy(bh)


def _mat(seed, m, n, decay):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, min(m, n))))
    V, _ = np.linalg.qr(rng.standard_normal((n, min(m, n))))
    s = decay ** np.arange(min(m, n))
    return (U * s) @ V.T, s


shapes = st.tuples(st.integers(6, 60), st.integers(6, 60)).filter(lambda t: min(t) >= 4)


@SLOW
@given(mn=shapes, seed=st.integers(0, 2 ** 31 - 1), q=st.integers(0, 3), p=st.integers(0, 12),
       decay=st.floats(0.3, 0.99), data=st.data())
def test_oracle_rsvd_invariants(mn, seed, q, p, decay, data):
    m, n = mn
    k = data.draw(st.integers(1, min(m, n) - 1))
    A, s_true = _mat(seed, m, n, decay)
    U, s, V, full = orc.rsvd(A, k, p=p, q=q, seed=seed, full=True)
    assert np.all(np.diff(s) <= 1e-12 * s[0]) and np.all(s >= 0)
    np.testing.assert_allclose(U.T @ U, np.eye(k), atol=1e-10)
    np.testing.assert_allclose(V.T @ V, np.eye(k), atol=1e-10)
    # interlacing: the sketch's values never exceed A's
    assert np.all(s <= s_true[:k] * (1 + 1e-10) + 1e-13)
    # sign rule: the largest-magnitude entry of each v_i is positive
    idx = np.argmax(np.abs(V), axis=0)
    assert np.all(V[idx, np.arange(k)] > 0)
    # U s V^T = Q Q^T A restricted to the top k: the residual is at least the
    # Eckart-Young optimum
    err = np.linalg.norm(A - (U * s) @ V.T, 2)
    assert err >= s_true[k] * (1 - 1e-9) - 1e-13


@SLOW
@given(mn=shapes, seed=st.integers(0, 2 ** 31 - 1), q=st.integers(0, 2), data=st.data())
def test_oracle_full_width_sketch_is_exact(mn, seed, q, data):
    m, n = mn
    k = data.draw(st.integers(1, min(m, n) - 1))
    A, s_true = _mat(seed, m, n, 0.8)
    _, s, _ = orc.rsvd(A, k, p=min(m, n), q=q, seed=seed)
    np.testing.assert_allclose(s, s_true[:k], rtol=1e-9, atol=1e-12)


@SLOW
@given(mn=shapes, seed=st.integers(0, 2 ** 31 - 1), data=st.data())
def test_oracle_exact_rank_is_recovered(mn, seed, data):
    m, n = mn
    r = data.draw(st.integers(1, min(m, n) - 2))
    k = data.draw(st.integers(r, min(m, n) - 1))
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    U, s, V = orc.rsvd(A, k, p=data.draw(st.integers(0, 5)), q=0, seed=seed)
    rel = np.linalg.norm(A - (U * s) @ V.T) / np.linalg.norm(A)
    assert rel < 1e-10


@SLOW
@given(mn=shapes, seed=st.integers(0, 2 ** 31 - 1), q=st.integers(1, 3), data=st.data())
def test_oracle_qr_and_lu_iterations_span_one_space(mn, seed, q, data):
    m, n = mn
    k = data.draw(st.integers(1, max(1, min(m, n) // 3)))
    A, _ = _mat(seed, m, n, 0.7)
    Qa, _, _ = orc.rqb(A, k, 2, q, seed, 0, "normal", "qr")
    Qb, _, _ = orc.rqb(A, k, 2, q, seed, 0, "normal", "lu")
    # principal angles between the two bases: ||Qa^T Qb|| singular values ~ 1
    c = np.linalg.svd(Qa.T @ Qb, compute_uv=False)
    assert c.min() > 1 - 1e-6


@SLOW
@given(mn=shapes, seed=st.integers(0, 2 ** 31 - 1))
def test_oracle_lu_factor(mn, seed):
    m, n = mn
    l = min(m, n)
    Y = np.random.default_rng(seed).standard_normal((m, l))
    Lf, U, piv = orc.lu_factor(Y)
    np.testing.assert_allclose(Lf @ U, Y, atol=1e-12 * max(1.0, np.abs(Y).max()) * l)
    assert np.all(np.abs(Lf) <= 1 + 1e-15)                  # partial pivoting bounds L
    Lt = Lf[piv]
    np.testing.assert_allclose(np.diag(Lt), 1.0)
    assert np.allclose(np.triu(Lt, 1), 0.0)
    assert len(set(piv.tolist())) == l and np.allclose(np.tril(U, -1), 0.0)


@SLOW
@given(mn=shapes, seed=st.integers(0, 2 ** 31 - 1), data=st.data())
def test_oracle_column_id(mn, seed, data):
    m, n = mn
    k = data.draw(st.integers(1, min(m, n) - 1))
    A, _ = _mat(seed, m, n, 0.6)
    C, Z, J = orid.interp_decomp(A, k)
    assert len(set(J.tolist())) == k
    np.testing.assert_allclose(Z[:, J], np.eye(k), atol=1e-12)
    np.testing.assert_array_equal(C, A[:, J])
    # column pivoting keeps |T| moderate on these well-conditioned leading blocks
    assert np.isfinite(Z).all()


@FAST
@given(x=st.lists(st.floats(-1e3, 1e3), min_size=1, max_size=40), tau=st.floats(0, 100))
def test_oracle_shrink_is_the_l1_prox(x, tau):
    x = np.array(x)
    y = orr.shrink(x, tau)
    assert np.all(np.abs(y) <= np.abs(x)) and np.all(y * x >= 0)
    # optimality: y minimises tau|y| + (y - x)^2 / 2, checked against nearby points
    f = lambda z: tau * np.abs(z) + 0.5 * (z - x) ** 2
    for d in (1e-3, -1e-3):
        assert np.all(f(y) <= f(y + d) + 1e-9)


@FAST
@given(seed=st.integers(0, 2 ** 63 - 1), sid=st.integers(0, 2 ** 31 - 1), n=st.integers(1, 9),
       l=st.integers(1, 9))
def test_oracle_philox_uniforms_are_open_interval(seed, sid, n, l):
    u = philox.uniforms(philox.raw_words(n, l, seed, sid))
    assert np.all(u > 0) and np.all(u < 1)
    om = philox.test_matrix(n, l, seed, sid, "rademacher")
    assert set(np.unique(om).tolist()) <= {-1.0, 1.0}


@FAST
@given(k=st.integers(8, 64), probs=st.lists(st.floats(0, 1), min_size=15, max_size=15), t1=st.floats(0.05, 1),
       t2=st.floats(0.05, 1))
def test_decision_cost_grows_with_tau(k, probs, t1, t2):
    """A larger confidence threshold never picks a cheaper pair."""
    from paper_1608_02148_amd import learned as lrn_gpu
    prob = np.array(probs)
    assume(prob.sum() > 0)
    prob = (prob / prob.sum())[None, :]
    lo, hi = sorted((t1, t2))
    a = lrn_gpu.decide(prob, [k], tau=lo)[0]
    b = lrn_gpu.decide(prob, [k], tau=hi)[0]
    qa, pa = lrn.class_pair(a)
    qb, pb = lrn.class_pair(b)
    assert lrn.pair_cost(k, qa, pa) <= lrn.pair_cost(k, qb, pb)
