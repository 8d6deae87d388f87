"""Learned choice of (q, p): labels, training on the GPU, checkpoints, and the
select-then-solve path.

The paper fixes only defaults (p = 10, q = 2, Sec. 3.6) and advises more
power iterations for slowly decaying spectra (Sec. 2.2).  Here a small network
reads the spectrum of a q = 0 sketch (rsvd_select) and picks the cheapest pair
(q, p) in {0..4} x {5, 10, 20} expected to reach the accuracy target; cost is
(2q + 2)(k + p), the passes over A times the sketch width.

Labels (training data).  For each matrix and each of the 15 pairs, one
batched solve (FP32 plain, the matrix's own Omega stream) gives U; the excess
error is ||(I - U U^T) A||_2 / sigma_{k+1} - 1 against the planted matrix
(whose spectrum and left factor are known exactly, synth.learned_data).  For
the rSVD's outputs U^T A = S V^T holds up to rounding, so this is the error
of A - U S V^T.  The spectral norm is the largest eigenvalue of
Sigma (I - W W^T) Sigma with W = U_true^T U (an r x k matrix), found by a
Krylov (Lanczos-type) iteration with full re-orthogonalisation and a
Rayleigh-Ritz step.  The label is the cheapest pair with excess error <= 1 %
(class 14 and "unreachable" when none is).

Training: Adam on mean cross-entropy through rsvd_mlp_train_step (the
library's own forward / backward / update kernels); torch only holds the
tensors and shuffles the sample order.

Checkpoint file: 64-byte header (magic b"RSVDMLP1", format version, parameter
count, Adam step, seed, training-set size, 8-byte hash of the training
features and labels), then theta, adam_m, adam_v as little-endian float32.
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


def save_checkpoint(path, tr, seed, n_train, digest):
    hdr = MAGIC + struct.pack("<IIIQQ", 1, L.MLP_PARAMS, tr.step_no, seed, n_train) + digest
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
    info = dict(step=hdr.step, seed=hdr.seed, n_train=hdr.n_train, digest=bytes(hdr.digest).hex())
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


def evaluate_arms(data, theta, seed=2148, reps=3, tau=DEFAULT_TAU, fixed=(4, 20)):
    """Three arms on one generated split (solves/s, fraction within 1 %):
    (i) FP32 plain at the paper's defaults q = 2, p = 10; (ii) FP32 plain at a
    fixed stronger pair; (iii) bf16 mixed precision with the learned (q, p),
    timed end to end (sketch features, network, planning, solve).  Excess
    errors are exact (residual_norms against the planted matrices)."""
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
                              theta=theta, tau=tau)
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


def main(argv=None):
    ap = argparse.ArgumentParser(description="train the (q, p) selector on generated matrices")
    ap.add_argument("--n-train", type=int, default=4096)
    ap.add_argument("--n-val", type=int, default=1024)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--out", default=DEFAULT_CHECKPOINT)
    ap.add_argument("--report", default=None)
    ap.add_argument("--dump", default=None, help="also save features, labels and error tables (.npz)")
    args = ap.parse_args(argv)
    from synth import learned_data as ld

    def log(msg):
        print(f"[selector] {msg}", file=sys.stderr, flush=True)

    out = {}
    sets = {}
    for split, count in (("train", args.n_train), ("val", args.n_val)):
        t0 = time.perf_counter()
        data = ld.build(count, split)
        torch.cuda.synchronize()
        log(f"{split}: {count} matrices generated in {time.perf_counter() - t0:.1f} s")
        t0 = time.perf_counter()
        tab = excess_table(data, log=log)
        ks = [int(x) for x in data["spec"]["k"]]
        lab, ok = labels_from_table(tab, ks)
        F = features(data)
        log(f"{split}: labels in {time.perf_counter() - t0:.1f} s; reachable {ok.mean():.4f}; "
            f"class histogram {np.bincount(lab, minlength=N_CLASSES).tolist()}")
        sets[split] = (F, torch.tensor(lab, device=F.device), tab, ok, ks)
        out[f"{split}_reachable"] = float(ok.mean())
        out[f"{split}_hist"] = np.bincount(lab, minlength=N_CLASSES).tolist()
        del data
        torch.cuda.empty_cache()
    F, y = sets["train"][0], sets["train"][1]
    Fv, yv = sets["val"][0], sets["val"][1]
    tr, hist = train(F, y, epochs=args.epochs, lr=args.lr, seed=args.seed, Fv=Fv, yv=yv, log=log)
    out["history"] = hist
    # validation: success rate and cost of the decision rule for several tau
    tabv, okv, ksv = sets["val"][2], sets["val"][3], sets["val"][4]
    prob, _ = api.mlp_forward(tr.theta, Fv)
    prob = prob.cpu().numpy()
    base = np.array([pair_cost(k, 7) for k in ksv]).sum()          # q = 2, p = 10
    for tau in (0.5, 0.7, DEFAULT_TAU, 0.9):
        pick = decide(prob, ksv, tau)
        err = tabv[np.arange(len(pick)), pick]
        cost = np.array([pair_cost(k, c) for k, c in zip(ksv, pick)]).sum()
        out[f"val_tau_{tau}"] = dict(success=float(np.mean(err <= TOL)),
                                     success_reachable=float(np.mean(err[okv] <= TOL)),
                                     cost_vs_default=float(cost / base))
        log(f"val tau={tau}: {out[f'val_tau_{tau}']}")
    if args.dump:
        np.savez(args.dump, **{f"{sp}_{name}": val for sp, (Fs, ys, tab, ok, ks) in sets.items()
                               for name, val in (("F", Fs.cpu().numpy()), ("y", ys.cpu().numpy()), ("tab", tab),
                                                 ("ok", ok), ("k", np.array(ks)))})
    save_checkpoint(args.out, tr, args.seed, args.n_train, data_hash(F, y))
    log(f"checkpoint written to {args.out}")
    if args.report:
        with open(args.report, "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
