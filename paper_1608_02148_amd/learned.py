"""Learned choice of (q, p): labels, training on the GPU, checkpoints, and the
select-then-solve path.

The paper fixes only defaults (p = 10, q = 2, Sec. 3.6) and advises more
power iterations for slowly decaying spectra (Sec. 2.2).  Here a small network
reads the spectrum of a q = 0 sketch (rsvd_select) and picks the cheapest pair
(q, p) in {0..4} x {5, 10, 20} expected to reach the accuracy target; cost is
(2q + 2)(k + p), the passes over A times the sketch width.

Labels (training data).  For each matrix and each of the 15 pairs, one
batched solve (FP32 plain, the matrix's own Omega stream) gives U; the excess
error is ||(I - U U^T) A||_2 / sigma_{k+1} - 1 with sigma_{k+1} from the
planted spectrum (synth.learned_data).  For the rSVD's outputs U^T A = S V^T
holds up to rounding, so this is the error of A - U S V^T.  The spectral norm
comes from a Krylov (Lanczos-type) iteration with full re-orthogonalisation
and a Rayleigh-Ritz step: on Sigma (I - W W^T) Sigma with W = U_true^T U when
the planted factors are Householder reflections (residual_norms), or on
E^T E with E = (I - U U^T) A from the stored matrices when they are dense
Haar factors (residual_norms_dense).  The label is the cheapest pair with
excess error <= 1 % (class 14 and "unreachable" when none is).

Pipeline (python -m paper_1608_02148_amd.learned ...):
  label --split train --count 40000 --lo L --hi H --dir D   shards of 4096
        matrices (dense Haar factors by default), each labelled and stored
        as D/<split>_<count>_<lo>_<hi>.npz (features, labels, error table);
  train --dir D --out selector.bin --report r.json           Adam on the
        train split, the device rule's threshold tau tuned on the validation
        split (the cheapest tau whose success reaches the fixed pair (4, 20)),
        test-split report, checkpoint.

Training: Adam on mean cross-entropy through rsvd_mlp_train_step (the
library's own forward / backward / update kernels); torch only holds the
tensors and shuffles the sample order.

Checkpoint file: 64-byte header (magic b"RSVDMLP1", format version, parameter
count, Adam step, seed, training-set size, 8-byte hash of the training
features and labels, f32 tau), then theta, adam_m, adam_v as little-endian
float32.
"""
import argparse
import ctypes
import hashlib
import json
import math
import os
import struct
import sys
import time

import numpy as np
import torch

from . import api
from . import lib as L

P_CHOICES = (5, 10, 20)
CLASS_PAIRS = [(q, p) for q in range(5) for p in P_CHOICES]
N_CLASSES = len(CLASS_PAIRS)
TOL = 0.01
FALLBACK_Q = 3
HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CHECKPOINT = os.path.join(HERE, "selector.bin")
MAGIC = b"RSVDMLP1"


def pair_cost(k, c):
    q, p = CLASS_PAIRS[c]
    return (2 * q + 2) * (k + p)


def classes_by_cost(k):
    return sorted(range(N_CLASSES), key=lambda c: (pair_cost(k, c), c))


# ------------------------------------------------------------------ exact errors

def _buckets(order, size):
    for i in range(0, len(order), size):
        yield order[i:i + size]


def residual_norms(data, Us, idx, krylov=40, bucket=256):
    """||(I - U U^T) A_b||_2 for the planted matrices b in idx (float64 numpy)."""
    if data.get("hh") is None:
        return residual_norms_dense(data, Us, idx, krylov)
    dev = data["A"][0].device
    spec = data["spec"]
    out = np.zeros(len(idx))
    pos = {b: i for i, b in enumerate(idx)}
    order = sorted(idx, key=lambda b: (min(spec["m"][b], spec["n"][b]), spec["m"][b]))
    g = torch.Generator(device=dev)
    g.manual_seed(12345)
    for grp in _buckets(order, bucket):
        B = len(grp)
        mx = int(max(spec["m"][b] for b in grp))
        rx = int(max(min(spec["m"][b], spec["n"][b]) for b in grp))
        kx = int(max(Us[b].shape[1] for b in grp))
        U = torch.zeros(B, mx, kx, dtype=torch.float64, device=dev)
        a1 = torch.zeros(B, mx, dtype=torch.float64, device=dev)
        a2 = torch.zeros_like(a1)
        sig = torch.zeros(B, rx, dtype=torch.float64, device=dev)
        for i, b in enumerate(grp):
            m, k = Us[b].shape
            r = len(data["sigma"][b])
            U[i, :m, :k] = Us[b].to(torch.float64)
            a1[i, :m], a2[i, :m] = data["hh"][b]
            sig[i, :r] = torch.as_tensor(data["sigma"][b], device=dev)
        # W = (U_true^T U) = (H(a2) H(a1) U)[:r]
        U = U - 2.0 * a1[:, :, None] * torch.bmm(a1[:, None, :], U)
        U = U - 2.0 * a2[:, :, None] * torch.bmm(a2[:, None, :], U)
        W = U[:, :rx, :].contiguous()
        mask = (sig > 0).to(torch.float64)
        W = W * mask[:, :, None]
        Wt = W.transpose(1, 2).contiguous()

        def apply(v):                      # Sigma (I - W W^T) Sigma v
            s = sig * v
            return sig * (s - torch.bmm(W, torch.bmm(Wt, s[:, :, None]))[:, :, 0])

        s = min(krylov, rx)
        Q = torch.zeros(B, rx, s, dtype=torch.float64, device=dev)
        MQ = torch.zeros_like(Q)
        v = torch.randn(B, rx, generator=g, device=dev, dtype=torch.float64) * mask
        v = v / v.norm(dim=1, keepdim=True).clamp_min(1e-300)
        for j in range(s):
            Q[:, :, j] = v
            w = apply(v)
            MQ[:, :, j] = w
            for _ in range(2):             # full re-orthogonalisation
                w = w - torch.bmm(Q[:, :, :j + 1], torch.bmm(Q[:, :, :j + 1].transpose(1, 2), w[:, :, None]))[:, :, 0]
            nrm = w.norm(dim=1, keepdim=True)
            v = torch.where(nrm > 1e-14 * sig[:, :1] ** 2, w / nrm.clamp_min(1e-300), torch.zeros_like(w))
        H = torch.bmm(Q.transpose(1, 2), MQ)
        H = 0.5 * (H + H.transpose(1, 2))
        lam = torch.linalg.eigvalsh(H)[:, -1].clamp_min(0.0)
        for i, b in enumerate(grp):
            out[pos[b]] = math.sqrt(float(lam[i]))
    return out


def residual_norms_dense(data, Us, idx, krylov=40, max_bytes=4 << 30):
    """||(I - U U^T) A_b||_2 from the stored matrices themselves (float64
    numpy), for inputs without known factors: E = P A with P = I - U U^T,
    the largest eigenvalue of E^T E by a Krylov iteration with full
    re-orthogonalisation (Lanczos-type, as residual_norms), matrices grouped
    by size into padded batches of at most max_bytes of float64 A."""
    A_list = data["A"]
    dev = A_list[0].device
    out = np.zeros(len(idx))
    pos = {b: i for i, b in enumerate(idx)}
    order = sorted(idx, key=lambda b: (A_list[b].shape[1], A_list[b].shape[0]))
    g = torch.Generator(device=dev)
    g.manual_seed(54321)
    i0 = 0
    while i0 < len(order):
        grp = [order[i0]]
        mx, nx = A_list[order[i0]].shape
        while i0 + len(grp) < len(order):
            b = order[i0 + len(grp)]
            m2, n2 = max(mx, A_list[b].shape[0]), max(nx, A_list[b].shape[1])
            if (len(grp) + 1) * m2 * n2 * 8 > max_bytes:
                break
            grp.append(b)
            mx, nx = m2, n2
        i0 += len(grp)
        B = len(grp)
        kx = int(max(Us[b].shape[1] for b in grp))
        A = torch.zeros(B, mx, nx, dtype=torch.float64, device=dev)
        U = torch.zeros(B, mx, kx, dtype=torch.float64, device=dev)
        mask = torch.zeros(B, nx, dtype=torch.float64, device=dev)
        for i, b in enumerate(grp):
            m, n = A_list[b].shape
            A[i, :m, :n] = A_list[b].to(torch.float64)
            U[i, :m, :Us[b].shape[1]] = Us[b].to(torch.float64)
            mask[i, :n] = 1.0
        At = A.transpose(1, 2).contiguous()
        Ut = U.transpose(1, 2).contiguous()

        def proj(w):                       # (I - U U^T) w
            return w - torch.bmm(U, torch.bmm(Ut, w[:, :, None]))[:, :, 0]

        def apply(v):                      # E^T E v, E = (I - U U^T) A
            w = proj(torch.bmm(A, v[:, :, None])[:, :, 0])
            return torch.bmm(At, proj(w)[:, :, None])[:, :, 0]

        s = min(krylov, nx)
        Q = torch.zeros(B, nx, s, dtype=torch.float64, device=dev)
        MQ = torch.zeros_like(Q)
        v = torch.randn(B, nx, generator=g, device=dev, dtype=torch.float64) * mask
        v = v / v.norm(dim=1, keepdim=True).clamp_min(1e-300)
        scale = torch.linalg.matrix_norm(A, ord="fro")[:, None] ** 2
        for j in range(s):
            Q[:, :, j] = v
            w = apply(v)
            MQ[:, :, j] = w
            for _ in range(2):
                w = w - torch.bmm(Q[:, :, :j + 1], torch.bmm(Q[:, :, :j + 1].transpose(1, 2), w[:, :, None]))[:, :, 0]
            nrm = w.norm(dim=1, keepdim=True)
            v = torch.where(nrm > 1e-14 * scale, w / nrm.clamp_min(1e-300), torch.zeros_like(w))
        H = torch.bmm(Q.transpose(1, 2), MQ)
        H = 0.5 * (H + H.transpose(1, 2))
        lam = torch.linalg.eigvalsh(H)[:, -1].clamp_min(0.0)
        for i, b in enumerate(grp):
            out[pos[b]] = math.sqrt(float(lam[i]))
        del A, At, U, Ut, Q, MQ
    return out


def excess_table(data, precision="plain", seed=2148, classes=None, log=None):
    """Excess error of every matrix under every class (N x 15, float64)."""
    n_mat = len(data["A"])
    ks = [int(x) for x in data["spec"]["k"]]
    classes = range(N_CLASSES) if classes is None else classes
    tab = np.full((n_mat, N_CLASSES), np.nan)
    for c in classes:
        q, p = CLASS_PAIRS[c]
        bt = api.Batch(data["A"], ks, p=p, q=q, seed=seed, precision=precision, compute_v=False, graph=False)
        bt.run()
        torch.cuda.synchronize()
        res = residual_norms(data, bt.U, list(range(n_mat)))
        sk1 = np.array([data["sigma"][b][ks[b]] for b in range(n_mat)])
        tab[:, c] = res / sk1 - 1.0
        if log:
            log(f"class {c} (q={q}, p={p}): fraction within {TOL:.0%}: {np.mean(tab[:, c] <= TOL):.4f}")
        bt.close()
        del bt
    return tab


def labels_from_table(tab, ks, tol=TOL):
    """(labels, reachable) from an excess-error table."""
    lab = np.full(len(ks), N_CLASSES - 1, dtype=np.int32)
    ok = np.zeros(len(ks), dtype=bool)
    for b, k in enumerate(ks):
        for c in classes_by_cost(k):
            if tab[b, c] <= tol:
                lab[b], ok[b] = c, True
                break
    return lab, ok


def features(data, precision="plain", seed=2148):
    ks = [int(x) for x in data["spec"]["k"]]
    bt = api.Batch(data["A"], ks, seed=seed, precision=precision, features=True, graph=False)
    bt.run()
    torch.cuda.synchronize()
    F = bt.features.clone()
    bt.close()
    return F


# ------------------------------------------------------------------ training

def train(F, y, epochs=300, lr=2e-3, batch=256, seed=7, Fv=None, yv=None, log=None):
    """Adam training of a fresh network on features F (N x 131) and labels y."""
    dev = F.device
    theta = api.mlp_init(seed=seed, device=dev)
    tr = api.MlpTrainer(theta, lr=lr)
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    N = F.shape[0]
    yi = y.to(torch.int32)
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(N, generator=g).to(dev)
        for i in range(0, N - batch + 1, batch):
            sel = perm[i:i + batch]
            tr.step(F[sel].contiguous(), yi[sel].contiguous())
        if log and (ep % 50 == 0 or ep == epochs - 1):
            _, cls = api.mlp_forward(theta, F)
            acc = float((cls == yi).float().mean())
            msg = dict(epoch=ep, loss=float(tr.loss), train_acc=round(acc, 4))
            if Fv is not None:
                _, cv = api.mlp_forward(theta, Fv)
                msg["val_acc"] = round(float((cv == yv.to(torch.int32)).float().mean()), 4)
            hist.append(msg)
            log(msg)
    return tr, hist


def data_hash(F, y):
    h = hashlib.sha256()
    h.update(F.detach().cpu().numpy().tobytes())
    h.update(y.detach().cpu().numpy().astype(np.int32).tobytes())
    return h.digest()[:8]


def save_checkpoint(path, tr, seed, n_train, digest, tau=0.0):
    hdr = MAGIC + struct.pack("<IIIQQ", 1, L.MLP_PARAMS, tr.step_no, seed, n_train) + digest
    hdr += struct.pack("<f", float(tau))
    hdr += b"\0" * (64 - len(hdr))
    with open(path, "wb") as f:
        f.write(hdr)
        for t in (tr.theta, tr.m, tr.v):
            f.write(t.detach().cpu().numpy().astype("<f4").tobytes())


def load_checkpoint(path=DEFAULT_CHECKPOINT, device="cuda", adam=False):
    """(theta tensor on device, header dict), read and checked by the
    library's rsvd_mlp_load; with adam=True also the Adam moments (theta,
    adam_m, adam_v).  Raises ValueError on a malformed file."""
    lib = L.load()
    hdr = L.MlpHeader()
    # check the file first (no device access), then copy it to the device
    h = ctypes.c_void_p()
    L.check(lib.rsvd_create(ctypes.byref(h), None), "rsvd_create")
    try:
        st = lib.rsvd_mlp_load(h, os.fsencode(path), None, None, None, ctypes.byref(hdr))
    finally:
        lib.rsvd_destroy(h)
    if st != 0:
        raise ValueError(f"{path}: not a usable selector checkpoint ({L.STATUS.get(st, st)})")
    theta = torch.empty(L.MLP_PARAMS, dtype=torch.float32, device=device)
    m = torch.empty_like(theta) if adam else None
    v = torch.empty_like(theta) if adam else None
    L.check(lib.rsvd_mlp_load(api.handle(theta.device), os.fsencode(path), theta.data_ptr(),
                              m.data_ptr() if adam else None, v.data_ptr() if adam else None,
                              ctypes.byref(hdr)), "rsvd_mlp_load")
    info = dict(step=hdr.step, seed=hdr.seed, n_train=hdr.n_train, digest=bytes(hdr.digest).hex(),
                tau=float(hdr.tau) if hdr.tau > 0 else None)
    return ((theta, m, v) if adam else theta), info


# ------------------------------------------------------------------ learned solve

# Pair c' dominates pair c when it has at least as many power iterations and
# at least as much oversampling; a pair that suffices is then very likely to
# be dominated only by pairs that suffice too.
def _dominates(a, b):
    return CLASS_PAIRS[a][0] <= CLASS_PAIRS[b][0] and CLASS_PAIRS[a][1] <= CLASS_PAIRS[b][1]


_LE = np.array([[_dominates(a, b) for b in range(N_CLASSES)] for a in range(N_CLASSES)], dtype=np.float64)
DEFAULT_TAU = 0.8


def decide(prob, ks, tau=DEFAULT_TAU):
    """Per-matrix class from the network's distribution over the cheapest
    sufficient pair: the cheapest class c whose estimated chance of sufficing,
    sum of P(label = L) over the pairs L that c dominates, reaches tau
    (class 14 when none does)."""
    cum = np.asarray(prob, dtype=np.float64) @ _LE
    pick = np.full(len(ks), N_CLASSES - 1, dtype=np.int32)
    for b, k in enumerate(ks):
        for c in classes_by_cost(int(k)):
            if cum[b, c] >= tau:
                pick[b] = c
                break
    return pick


def choose(theta, As, ks, seed=2148, precision="plain", tau=DEFAULT_TAU):
    """Per-matrix (q, p) from the network (rsvd_select features, then decide());
    without a network (theta None) the fixed fallback q = 3, p = 10."""
    n = len(As)
    if theta is None:
        return np.full(n, FALLBACK_Q, dtype=np.int32), np.full(n, 10, dtype=np.int32)
    qs, ps, _ = api.select(As, ks, theta, seed=seed, precision=precision, tau=tau)
    return qs, ps


def load_or_fallback(path=DEFAULT_CHECKPOINT, device="cuda"):
    """The trained network, or None (fixed q = 3 fallback) when the file is
    absent or malformed."""
    try:
        return load_checkpoint(path, device)[0]
    except (OSError, ValueError):
        return None


def _timed_batch(data, ks, reps, **kw):
    """Build a graph-captured batch, warm it up, time `reps` replays (ms each)."""
    bt = api.Batch(data["A"], ks, compute_v=False, graph=True, **kw)
    bt.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        bt.run()
    torch.cuda.synchronize()
    return bt, (time.perf_counter() - t0) * 1e3 / reps


def evaluate_arms(data, theta, seed=2148, reps=3, tau=DEFAULT_TAU, fixed=(4, 20), tau_graph=None):
    """Three arms on one generated split (solves/s, fraction within 1 %):
    (i) FP32 plain at the paper's defaults q = 2, p = 10; (ii) FP32 plain at a
    fixed stronger pair; (iii) bf16 mixed precision with the learned (q, p),
    timed end to end (sketch features, network, planning, solve).  Excess
    errors are exact (residual_norms against the planted matrices).  tau:
    threshold of the host route (decide); tau_graph: of the device rule
    (default tau)."""
    n_mat = len(data["A"])
    ks = [int(x) for x in data["spec"]["k"]]
    sk1 = np.array([data["sigma"][b][ks[b]] for b in range(n_mat)])

    def success(bt):
        err = residual_norms(data, bt.U, list(range(n_mat))) / sk1 - 1.0
        return err

    out = {}
    work = None
    for name, (q, p) in (("fp32_default_q2_p10", (2, 10)), (f"fp32_fixed_q{fixed[0]}_p{fixed[1]}", fixed)):
        bt, ms = _timed_batch(data, ks, reps, p=p, q=q, seed=seed)
        err = success(bt)
        out[name] = dict(ms=ms, solves_per_s=n_mat / ms * 1e3, errors=err)
        bt.close()
        if work is None or bt.work.numel() > work.numel():
            work = bt.work          # reused by the learned arms (p <= 20, q <= 4: no larger)
        del bt
    # learned on the device (one graph: q = 0 sketches, features, network,
    # choice of q, then the solves from those sketches; p = 20 for every
    # matrix, which covers every class of the label set at the chosen q)
    for name, prec in (("fp32_learned_graph", "plain"), ("bf16_learned_graph", "bf16_mixed")):
        bt, ms = _timed_batch(data, ks, reps, p=P_CHOICES[-1], seed=seed, precision=prec, learned=True,
                              theta=theta, tau=tau if tau_graph is None else tau_graph)
        q = bt.choices()
        err = success(bt)
        out[name] = dict(ms=ms, solves_per_s=n_mat / ms * 1e3, errors=err,
                         q_hist=np.bincount(q, minlength=5).tolist())
        bt.close()
        del bt
    # learned through the host: select (features + network) returns (q, p),
    # then a batch is planned with them; selection and planning are timed too
    for name, prec in (("fp32_learned", "plain"), ("bf16_learned", "bf16_mixed")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            qs, ps = choose(theta, data["A"], ks, seed=seed, precision=prec, tau=tau)
        torch.cuda.synchronize()
        select_ms = (time.perf_counter() - t0) * 1e3 / reps
        t0 = time.perf_counter()
        bt = api.Batch(data["A"], ks, seed=seed, precision=prec, qs=qs, ps=ps, compute_v=False, graph=False,
                       work=work)
        plan_ms = (time.perf_counter() - t0) * 1e3
        bt.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            bt.run()
        torch.cuda.synchronize()
        solve_ms = (time.perf_counter() - t0) * 1e3 / reps
        err = success(bt)
        total = select_ms + plan_ms + solve_ms
        out[name] = dict(ms=total, select_ms=select_ms, plan_ms=plan_ms, solve_ms=solve_ms,
                         solves_per_s=n_mat / total * 1e3, errors=err,
                         q_hist=np.bincount(qs, minlength=5).tolist(),
                         p_hist={int(v): int(np.sum(ps == v)) for v in P_CHOICES})
        bt.close()
    return out


def device_q_rule(prob, tau):
    """The choice of q that rsvd_batch_create_learned makes on the device for
    solves at p = 20 (every class covered by its q): the fewest q whose
    classes hold mass >= tau, else 4 (tau <= 0: the most probable class)."""
    prob = np.asarray(prob, dtype=np.float64)
    if tau <= 0:
        return np.argmax(prob, axis=1) // len(P_CHOICES)
    cum = np.cumsum(prob.reshape(len(prob), -1, len(P_CHOICES)).sum(axis=2), axis=1)
    hit = cum >= tau
    return np.where(hit.any(axis=1), np.argmax(hit, axis=1), 4)


def label_shard(count, split, lo, hi, factors):
    """Features (float32 numpy, (hi - lo) x 131), labels, error table,
    reachability and target ranks of matrices lo..hi-1 of a split of `count`
    generated matrices."""
    from synth import learned_data as ld
    data = ld.build_range(count, split, lo, hi, factors=factors)
    tab = excess_table(data)
    ks = np.array([int(x) for x in data["spec"]["k"]])
    lab, ok = labels_from_table(tab, ks)
    F = features(data).cpu().numpy()
    del data
    torch.cuda.empty_cache()
    return dict(F=F, y=lab, tab=tab, ok=ok, k=ks)


def _log(msg):
    print(f"[selector] {msg}", file=sys.stderr, flush=True)


def cmd_label(args):
    """Label shards of a split and store them as .npz files (one per shard)."""
    os.makedirs(args.dir, exist_ok=True)
    hi_all = args.count if args.hi is None else min(args.hi, args.count)
    for lo in range(args.lo, hi_all, args.shard):
        hi = min(hi_all, lo + args.shard)
        t0 = time.perf_counter()
        d = label_shard(args.count, args.split, lo, hi, args.factors)
        np.savez(os.path.join(args.dir, f"{args.split}_{args.count}_{lo:06d}_{hi:06d}.npz"), **d)
        _log(f"{args.split} [{lo}, {hi}) of {args.count}: {time.perf_counter() - t0:.1f} s, reachable "
             f"{d['ok'].mean():.4f}")


def _load_split(dirname, split):
    parts = sorted(f for f in os.listdir(dirname) if f.startswith(split + "_") and f.endswith(".npz"))
    if not parts:
        return None
    ds = [np.load(os.path.join(dirname, f)) for f in parts]
    return {key: np.concatenate([d[key] for d in ds]) for key in ("F", "y", "tab", "ok", "k")}


def cmd_train(args):
    """Train on labelled shards, tune the device rule's threshold on the
    validation split, evaluate on the test split, write the checkpoint."""
    sets = {sp: _load_split(args.dir, sp) for sp in ("train", "val", "test")}
    out = {f"n_{sp}": (0 if d is None else int(len(d["y"]))) for sp, d in sets.items()}
    for sp, d in sets.items():
        if d is not None:
            out[f"{sp}_reachable"] = float(d["ok"].mean())
            out[f"{sp}_hist"] = np.bincount(d["y"], minlength=N_CLASSES).tolist()
    dev = torch.device("cuda")
    F = torch.tensor(sets["train"]["F"], device=dev)
    y = torch.tensor(sets["train"]["y"], device=dev)
    Fv = torch.tensor(sets["val"]["F"], device=dev)
    yv = torch.tensor(sets["val"]["y"], device=dev)
    tr, hist = train(F, y, epochs=args.epochs, lr=args.lr, seed=args.seed, Fv=Fv, yv=yv, log=_log)
    out["history"] = hist

    def rule_stats(sp, tau):
        d = sets[sp]
        prob = api.mlp_forward(tr.theta, torch.tensor(d["F"], device=dev))[0].cpu().numpy()
        q = device_q_rule(prob, tau)
        err = d["tab"][np.arange(len(q)), 3 * q + 2]               # solves at p = 20
        cost = np.array([pair_cost(int(k), 3 * int(qq) + 2) for k, qq in zip(d["k"], q)]).sum()
        fixed = np.array([pair_cost(int(k), N_CLASSES - 1) for k in d["k"]]).sum()
        return dict(success=float(np.mean(err <= TOL)), success_reachable=float(np.mean(err[d["ok"]] <= TOL)),
                    cost_vs_fixed_q4_p20=float(cost / fixed), q_hist=np.bincount(q, minlength=5).tolist())

    # threshold of the device rule: the cheapest tau whose validation success
    # reaches that of the fixed pair (q, p) = (4, 20)
    target = float(np.mean(sets["val"]["tab"][:, N_CLASSES - 1] <= TOL))
    out["val_fixed_q4_p20_success"] = target
    best = None
    for tau in np.round(np.arange(0.50, 1.0, 0.01), 2):
        st = rule_stats("val", float(tau))
        out[f"val_tau_{tau:.2f}"] = st
        if st["success"] >= target and (best is None or st["cost_vs_fixed_q4_p20"] < best[1]["cost_vs_fixed_q4_p20"]):
            best = (float(tau), st)
    tau = best[0] if best else 0.99
    out["tau"] = tau
    _log(f"tau {tau}: validation {best[1] if best else None} (fixed (4, 20): {target:.4f})")
    if sets["test"] is not None:
        tab = sets["test"]["tab"]
        out["test_fixed_q4_p20_success"] = float(np.mean(tab[:, N_CLASSES - 1] <= TOL))
        out["test_fixed_q2_p10_success"] = float(np.mean(tab[:, 7] <= TOL))
        out["test_learned"] = rule_stats("test", tau)
        _log(f"test: learned {out['test_learned']}, fixed (4, 20) {out['test_fixed_q4_p20_success']:.4f}, "
             f"(2, 10) {out['test_fixed_q2_p10_success']:.4f}")
    save_checkpoint(args.out, tr, args.seed, len(sets["train"]["y"]), data_hash(F, y), tau)
    _log(f"checkpoint written to {args.out}")
    if args.report:
        with open(args.report, "w") as f:
            json.dump(out, f, indent=1)


def main(argv=None):
    ap = argparse.ArgumentParser(description="label generated matrices and train the (q, p) selector")
    sub = ap.add_subparsers(dest="cmd", required=True)
    lb = sub.add_parser("label", help="label shards of a split into .npz files")
    lb.add_argument("--split", required=True, choices=("train", "val", "test"))
    lb.add_argument("--count", type=int, required=True, help="size of the whole split")
    lb.add_argument("--lo", type=int, default=0)
    lb.add_argument("--hi", type=int, default=None)
    lb.add_argument("--shard", type=int, default=4096)
    lb.add_argument("--factors", default="haar", choices=("haar", "householder"))
    lb.add_argument("--dir", required=True)
    tn = sub.add_parser("train", help="train on labelled shards and write the checkpoint")
    tn.add_argument("--dir", required=True)
    tn.add_argument("--epochs", type=int, default=200)
    tn.add_argument("--lr", type=float, default=2e-3)
    tn.add_argument("--seed", type=int, default=7)
    tn.add_argument("--out", default=DEFAULT_CHECKPOINT)
    tn.add_argument("--report", default=None)
    args = ap.parse_args(argv)
    if args.cmd == "label":
        cmd_label(args)
    else:
        cmd_train(args)


if __name__ == "__main__":
    main()
