"""C ABI checks that need no GPU: the library loads, exports every symbol the
public header declares, and rejects bad arguments before any launch."""
import ctypes
import os
import re

import pytest

from paper_1608_02148_amd import lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rsvd_mi355x.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rsvd_\w+|rpca_\w+|rrpca_\w+|rid_\w+|rcur_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return L.load()


def test_library_exports_every_declared_symbol(lib):
    names = header_functions()
    assert len(names) >= 16
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(L.EXPORTED)


def test_struct_layouts_match_header():
    assert ctypes.sizeof(L.Params) == 40
    assert ctypes.sizeof(L.Info) == 24
    assert ctypes.sizeof(L.BatchDesc) == 104


def test_default_params_are_the_papers(lib):
    prm = L.Params()
    lib.rsvd_default_params(ctypes.byref(prm))
    assert (prm.p, prm.q, prm.sdist, prm.precision) == (10, 2, 0, 0)


def test_status_strings(lib):
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.rsvd_status_string(code).decode() == L.STATUS[code]


@pytest.fixture(scope="module")
def handle(lib):
    h = ctypes.c_void_p()
    assert lib.rsvd_create(ctypes.byref(h), None) == 0
    yield h
    lib.rsvd_destroy(h)


def _ws(lib, h, dtype, m, n, k, p=10, q=2, **kw):
    prm = L.Params()
    lib.rsvd_default_params(ctypes.byref(prm))
    prm.p, prm.q = p, q
    for key, v in kw.items():
        setattr(prm, key, v)
    out = ctypes.c_size_t(0)
    st = lib.rsvd_workspace_size(h, dtype, m, n, k, ctypes.byref(prm), ctypes.byref(out))
    return st, out.value


@pytest.mark.parametrize("m,n,k,p,q,want", [
    (100, 50, 0, 10, 2, -1),     # k < 1
    (100, 50, 50, 10, 2, -1),    # k >= min(m, n)
    (100, 50, 60, 10, 2, -1),
    (0, 50, 5, 10, 2, -1),
    (100, 50, 5, -1, 2, -1),     # p < 0
    (100, 50, 5, 10, -1, -1),    # q < 0
    (100000, 5000, 240, 20, 2, -2),   # l = 260 exceeds the single-solve limit
    (100000, 5000, 200, 20, 2, 0),    # l = 220: blocked Cholesky, Jacobi in global memory
    (100, 50, 5, 10, 2, 0),
    (100, 50, 45, 10, 2, 0),     # l clamped to min(m, n) = 50
])
def test_workspace_argument_rules(lib, handle, m, n, k, p, q, want):
    st, nbytes = _ws(lib, handle, L.RSVD_F32, m, n, k, p, q)
    assert st == want
    if want == 0:
        assert nbytes > 0 and nbytes % 256 == 0


def test_bad_dtype_and_mode_are_unsupported(lib, handle):
    assert _ws(lib, handle, 7, 100, 50, 5)[0] == -2
    assert _ws(lib, handle, L.RSVD_F32, 100, 50, 5, sdist=9)[0] == -1


def test_run_rejects_null_and_small_workspace_before_launch(lib, handle):
    prm = L.Params()
    lib.rsvd_default_params(ctypes.byref(prm))
    fake = ctypes.c_void_p(256)        # never dereferenced: checks fail first
    S = ctypes.c_void_p(512)
    # NULL A
    assert lib.rsvd_run(handle, L.RSVD_F32, 100, 50, None, 50, 5, ctypes.byref(prm),
                        None, 0, S, None, 0, fake, 1 << 30, None) == -1
    # lda < n
    assert lib.rsvd_run(handle, L.RSVD_F32, 100, 50, fake, 49, 5, ctypes.byref(prm),
                        None, 0, S, None, 0, fake, 1 << 30, None) == -1
    # workspace too small
    assert lib.rsvd_run(handle, L.RSVD_F32, 100, 50, fake, 50, 5, ctypes.byref(prm),
                        None, 0, S, None, 0, fake, 16, None) == -1
    # misaligned workspace
    assert lib.rsvd_run(handle, L.RSVD_F32, 100, 50, fake, 50, 5, ctypes.byref(prm),
                        None, 0, S, None, 0, ctypes.c_void_p(264), 1 << 30, None) == -1
    # NULL S
    assert lib.rsvd_run(handle, L.RSVD_F32, 100, 50, fake, 50, 5, ctypes.byref(prm),
                        None, 0, None, None, 0, fake, 1 << 30, None) == -1
    # ldu < k
    assert lib.rsvd_run(handle, L.RSVD_F32, 100, 50, fake, 50, 5, ctypes.byref(prm),
                        fake, 4, S, None, 0, fake, 1 << 30, None) == -1
    # PCA needs rotation and eigvals
    assert lib.rpca_run(handle, L.RSVD_F32, 100, 50, fake, 50, 5, 1, ctypes.byref(prm),
                        None, 5, S, None, None, 0, None, fake, 1 << 30, None) == -1


def test_precision_mode_unknown_is_rejected(lib, handle):
    assert _ws(lib, handle, L.RSVD_F32, 100, 50, 5, precision=5)[0] == -2


def _descs(shapes, U=True):
    arr = (L.BatchDesc * len(shapes))()
    for b, (m, n, k) in enumerate(shapes):
        d = arr[b]
        d.A, d.lda, d.m, d.n, d.k, d.stream_id = 4096 * (b + 1), n, m, n, k, b
        d.U, d.ldu = (1 << 20, k) if U else (None, 0)
        d.S, d.V, d.ldv, d.info = 1 << 21, 1 << 22, k, None
        d.features, d.q, d.p = None, -1, -1
    return arr


def _create(lib, handle, shapes, dtype=L.RSVD_F32, flags=0, descs=None, **kw):
    prm = L.Params()
    lib.rsvd_default_params(ctypes.byref(prm))
    for key, v in kw.items():
        setattr(prm, key, v)
    descs = descs if descs is not None else _descs(shapes)
    b = ctypes.c_void_p()
    nbytes = ctypes.c_size_t(0)
    st = lib.rsvd_batch_create(handle, dtype, len(shapes), descs, ctypes.byref(prm), flags, ctypes.byref(b),
                               ctypes.byref(nbytes))
    return st, b, nbytes.value


def test_batch_create_is_host_only_and_sizes_the_workspace(lib, handle):
    """Planning a batch records its steps on the host; nothing is launched."""
    shapes = [(300, 200, 10), (1000, 100, 50), (64, 40, 1), (700, 1300, 118)]
    st, b, nbytes = _create(lib, handle, shapes, flags=L.BATCH_GRAPH | L.BATCH_STAMPS)
    assert st == 0 and b.value
    singles = sum(_ws(lib, handle, L.RSVD_F32, m, n, k)[1] for m, n, k in shapes)
    assert nbytes % 256 == 0
    # per-matrix workspaces (no split partials) plus the launch tables
    assert nbytes > 2 * 8 * len(shapes)
    assert nbytes < 2 * singles + (1 << 24)
    # run before bind, stamps before bind: invalid
    assert lib.rsvd_batch_run(b) == -1
    assert lib.rsvd_batch_stamps(b, ctypes.c_void_p(8), None) == -1
    # bind with a too small or misaligned buffer fails before any copy
    assert lib.rsvd_batch_bind(b, ctypes.c_void_p(256), nbytes - 1) == -1
    assert lib.rsvd_batch_bind(b, ctypes.c_void_p(264), nbytes) == -1
    assert lib.rsvd_batch_destroy(b) == 0


@pytest.mark.parametrize("shapes,want", [
    ([(100, 50, 50)], -1),                    # k >= min(m, n)
    ([(100, 50, 5), (100, 50, 0)], -1),       # k < 1 in a later entry
    ([(400, 300, 125)], -2),                  # l = 135 > RSVD_MAX_L
    ([(100, 50, 5)] * 3, 0),
])
def test_batch_argument_rules(lib, handle, shapes, want):
    st, b, _ = _create(lib, handle, shapes)
    assert st == want
    lib.rsvd_batch_destroy(b)


def test_batch_rejects_mixed_outputs_flags_and_lda(lib, handle):
    shapes = [(100, 50, 5), (120, 60, 6)]
    d = _descs(shapes)
    d[1].U = None
    assert _create(lib, handle, shapes, descs=d)[0] == -1      # U given for some entries only
    d = _descs(shapes)
    d[0].lda = 49
    assert _create(lib, handle, shapes, descs=d)[0] == -1
    d = _descs(shapes)
    d[1].S = None
    assert _create(lib, handle, shapes, descs=d)[0] == -1
    assert _create(lib, handle, shapes, flags=8)[0] == -1
    assert _create(lib, handle, shapes, dtype=L.RSVD_F64, precision=1)[0] == -2
    prm = L.Params()
    lib.rsvd_default_params(ctypes.byref(prm))
    b = ctypes.c_void_p()
    nbytes = ctypes.c_size_t(0)
    assert lib.rsvd_batch_create(handle, L.RSVD_F32, 0, _descs(shapes), ctypes.byref(prm), 0, ctypes.byref(b),
                                 ctypes.byref(nbytes)) == -1


def test_batch_feature_and_own_qp_rules(lib, handle):
    shapes = [(300, 200, 10), (1000, 100, 50)]
    d = _descs(shapes)
    # features mode needs a features pointer per matrix; S is not needed
    assert _create(lib, handle, shapes, flags=L.BATCH_FEATURES, descs=d)[0] == -1
    for b in range(2):
        d[b].features, d[b].S = 1 << 23, None
    st, b, nbytes = _create(lib, handle, shapes, flags=L.BATCH_FEATURES, descs=d)
    assert st == 0 and nbytes > 0
    lib.rsvd_batch_destroy(b)
    # own q / p: taken from each desc and checked like params
    d = _descs(shapes)
    d[0].q, d[0].p, d[1].q, d[1].p = 3, 5, 0, 20
    st, b, _ = _create(lib, handle, shapes, flags=L.BATCH_OWN_QP, descs=d)
    assert st == 0
    lib.rsvd_batch_destroy(b)
    d[1].q = -1
    assert _create(lib, handle, shapes, flags=L.BATCH_OWN_QP, descs=d)[0] == -1
    d[1].q = 1
    d[0].q, d[0].p = 1, 125                # l = min(135, 200) > RSVD_MAX_L
    assert _create(lib, handle, shapes, flags=L.BATCH_OWN_QP, descs=d)[0] == -2


def _create_learned(lib, handle, shapes, descs=None, flags=L.BATCH_GRAPH, tau=0.8, **prm_kw):
    prm = L.Params()
    lib.rsvd_default_params(ctypes.byref(prm))
    for key, v in prm_kw.items():
        setattr(prm, key, v)
    descs = descs if descs is not None else _descs(shapes)
    b = ctypes.c_void_p()
    nbytes = ctypes.c_size_t(0)
    st = lib.rsvd_batch_create_learned(handle, L.RSVD_F32, len(shapes), descs, ctypes.byref(prm), None,
                                       ctypes.c_float(tau), flags, ctypes.byref(b), ctypes.byref(nbytes))
    return st, b, nbytes.value


def test_learned_batch_rules(lib, handle):
    """Learned batches: host-only planning; p bounded by the largest class's
    oversampling; flags limited to graph and stamps; like rsvd_batch_create
    otherwise."""
    shapes = [(300, 200, 10), (1000, 100, 50), (700, 1300, 108), (64, 40, 1)]
    st, b, nbytes = _create_learned(lib, handle, shapes, p=20)
    assert st == 0 and nbytes > 0
    # two workspaces per matrix (sketch phase and solve) exceed the plain batch
    st2, b2, plain = _create(lib, handle, shapes)
    assert st2 == 0 and nbytes > plain
    assert lib.rsvd_batch_run(b) == -1                       # not bound
    assert lib.rsvd_batch_choices(b, ctypes.c_void_p(8)) == -1
    assert lib.rsvd_batch_choices(b2, ctypes.c_void_p(8)) == -1   # not a learned batch
    lib.rsvd_batch_destroy(b)
    lib.rsvd_batch_destroy(b2)
    assert _create_learned(lib, handle, shapes, p=21)[0] == -1
    assert _create_learned(lib, handle, shapes, p=-1)[0] == -1
    assert _create_learned(lib, handle, shapes, tau=float("nan"))[0] == -1
    assert _create_learned(lib, handle, shapes, tau=1.5)[0] == -1
    assert _create_learned(lib, handle, shapes, flags=L.BATCH_FEATURES)[0] == -1
    assert _create_learned(lib, handle, shapes, flags=L.BATCH_OWN_QP)[0] == -1
    assert _create_learned(lib, handle, [(100, 50, 50)])[0] == -1
    d = _descs(shapes)
    d[2].S = None
    assert _create_learned(lib, handle, shapes, descs=d)[0] == -1
    st, b, _ = _create_learned(lib, handle, shapes, precision=1, p=10)
    assert st == 0
    lib.rsvd_batch_destroy(b)


def test_select_workspace_is_host_only(lib, handle):
    shapes = [(300, 200, 10), (4000, 1000, 64)]
    prm = L.Params()
    lib.rsvd_default_params(ctypes.byref(prm))
    nbytes = ctypes.c_size_t(0)
    assert lib.rsvd_select_workspace_size(handle, L.RSVD_F32, 2, _descs(shapes), ctypes.byref(prm),
                                          ctypes.byref(nbytes)) == 0
    assert nbytes.value >= 2 * 131 * 4
    assert lib.rsvd_select(handle, L.RSVD_F32, 2, _descs(shapes), ctypes.byref(prm), None, 0.8, None, None,
                           None, ctypes.c_void_p(256), nbytes.value) == -1


def test_numpy_descriptor_layout_matches_the_struct():
    import numpy as np
    from paper_1608_02148_amd import api
    dt = api._desc_dtype()
    assert dt.itemsize == ctypes.sizeof(L.BatchDesc)
    d = np.zeros(2, dtype=dt)
    d["A"], d["lda"], d["m"], d["n"], d["k"], d["stream_id"] = [11, 12], [5, 6], [300, 400], [200, 100], [7, 8], [3, 4]
    d["U"], d["ldu"], d["S"], d["V"], d["ldv"] = [21, 22], [7, 8], [31, 32], [41, 42], [7, 8]
    d["info"], d["features"], d["q"], d["p"] = [51, 52], [61, 62], [2, 3], [10, 20]
    c = (L.BatchDesc * 2).from_buffer_copy(d.tobytes())
    assert (c[1].A, c[1].lda, c[1].m, c[1].n, c[1].k, c[1].stream_id) == (12, 6, 400, 100, 8, 4)
    assert (c[1].U, c[1].ldu, c[1].S, c[1].V, c[1].ldv) == (22, 8, 32, 42, 8)
    assert (c[1].info, c[1].features, c[1].q, c[1].p) == (52, 62, 3, 20)


def test_single_solve_width_limit(lib, handle):
    """Single solves take sketch widths up to RSVD_MAX_L_SINGLE = 256 (batches
    stay at RSVD_MAX_L = 128); the wider workspace includes the blocked
    Cholesky's scratch and the Jacobi matrix."""
    st, wide = _ws(lib, handle, L.RSVD_F32, 3000, 1000, 200)
    assert st == 0
    st, narrow = _ws(lib, handle, L.RSVD_F32, 3000, 1000, 100)
    assert st == 0 and wide > narrow + 7 * 128 * 128 * 8
    assert _ws(lib, handle, L.RSVD_F32, 3000, 1000, 236, p=20)[0] == 0      # l = 256
    assert _ws(lib, handle, L.RSVD_F32, 3000, 1000, 237, p=20)[0] == -2     # l = 257
    assert _create(lib, handle, [(3000, 1000, 200)])[0] == -2          # batches: l <= 128


def _checkpoint_bytes(version=1, nparams=13583, values=None, magic=b"RSVDMLP1"):
    import struct
    import numpy as np
    hdr = magic + struct.pack("<IIIQQ", version, nparams, 77, 5, 8192) + bytes(range(8))
    hdr += b"\0" * (64 - len(hdr))
    vals = np.zeros(3 * 13583, dtype="<f4") if values is None else values
    return hdr + vals.astype("<f4").tobytes()


def test_mlp_load_checks_the_file_without_a_device(lib, handle, tmp_path):
    """rsvd_mlp_load reads and checks the whole checkpoint before any device
    access: theta = NULL checks only; a bad file fails with theta set too."""
    import numpy as np
    good = tmp_path / "good.bin"
    good.write_bytes(_checkpoint_bytes(values=np.linspace(-1, 1, 3 * 13583)))
    hdr = L.MlpHeader()
    assert lib.rsvd_mlp_load(handle, str(good).encode(), None, None, None, ctypes.byref(hdr)) == 0
    assert (hdr.version, hdr.params, hdr.step, hdr.seed, hdr.n_train) == (1, 13583, 77, 5, 8192)
    assert bytes(hdr.digest) == bytes(range(8))
    fake = ctypes.c_void_p(16)          # never dereferenced: every case below fails first
    cases = {
        "absent.bin": None,
        "magic.bin": _checkpoint_bytes(magic=b"NOTMLP01"),
        "version.bin": _checkpoint_bytes(version=2),
        "count.bin": _checkpoint_bytes(nparams=100),
        "short.bin": _checkpoint_bytes()[:-4],
        "long.bin": _checkpoint_bytes() + b"\0",
        "header.bin": b"RSVDMLP1\x01",
    }
    want = {"absent.bin": -1, "magic.bin": -2, "version.bin": -2, "count.bin": -2, "short.bin": -1,
            "long.bin": -1, "header.bin": -1}
    for name, raw in cases.items():
        p = tmp_path / name
        if raw is not None:
            p.write_bytes(raw)
        assert lib.rsvd_mlp_load(handle, str(p).encode(), fake, None, None, None) == want[name], name
    for bad in (np.nan, np.inf):
        vals = np.zeros(3 * 13583)
        vals[2 * 13583 + 5] = bad                 # in adam_v
        p = tmp_path / "nonfinite.bin"
        p.write_bytes(_checkpoint_bytes(values=vals))
        assert lib.rsvd_mlp_load(handle, str(p).encode(), fake, fake, fake, None) == -1
    assert lib.rsvd_mlp_load(handle, None, fake, None, None, None) == -1
    assert lib.rsvd_mlp_load(None, str(good).encode(), None, None, None, None) == -1
    assert lib.rsvd_mlp_load(handle, str(good).encode(), None, fake, None, None) == -1


def test_committed_checkpoint_passes_the_library_check(lib, handle):
    from paper_1608_02148_amd import learned
    hdr = L.MlpHeader()
    assert lib.rsvd_mlp_load(handle, learned.DEFAULT_CHECKPOINT.encode(), None, None, None,
                             ctypes.byref(hdr)) == 0
    assert hdr.params == 13583 and hdr.step > 0 and hdr.n_train > 0


def test_power_scheme_rules(lib, handle):
    """LU normalisation: l <= 128 and single solves only; unknown schemes are
    invalid (all checked before any launch)."""
    st, with_lu = _ws(lib, handle, L.RSVD_F32, 5000, 1000, 100, 20, 2, scheme=1)
    assert st == 0 and with_lu > _ws(lib, handle, L.RSVD_F32, 5000, 1000, 100, 20, 2)[1]   # pivot lists
    assert _ws(lib, handle, L.RSVD_F32, 5000, 1000, 120, 20, 2, scheme=1)[0] == -2
    assert _ws(lib, handle, L.RSVD_F32, 5000, 1000, 10, 10, 2, scheme=2)[0] == -1
    prm = L.Params()
    lib.rsvd_default_params(ctypes.byref(prm))
    prm.scheme = 1
    d = (L.BatchDesc * 1)()
    d[0].A, d[0].lda, d[0].m, d[0].n, d[0].k = 256, 100, 300, 100, 10
    d[0].S = 512
    b = ctypes.c_void_p()
    nbytes = ctypes.c_size_t()
    assert lib.rsvd_batch_create(handle, L.RSVD_F32, 1, d, ctypes.byref(prm), 0, ctypes.byref(b),
                                 ctypes.byref(nbytes)) == -2
