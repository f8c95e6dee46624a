"""Training driver of the learned start proposer (this library's addition).

Data: seeded synthetic 1920x1088 sequences (synth.training_sequence: objects
with velocities Laplace(0, 8) x Laplace(0, 4) clipped to +-31, a panning
background), 40 sequences x 50 frames = 2000 frames by default.  Labels: the
library's own full search at range +-31 on the GPU.  Training: minibatches of
frame pairs, Adam, cosine learning-rate decay, all on the GPU through the C ABI
(me_proposer_train_step).  Output: an .npz checkpoint (weights, Adam moments,
step, configuration; no pickled objects).

    python -m paper_0806_0689_amd.train --out paper_0806_0689_amd/weights/proposer.npz
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "proposer.npz")


def _make(args):
    q, frames, held_out = args
    from synth import training_sequence
    return training_sequence(q, frames=frames, held_out=held_out)


def generate(qs, frames, held_out=False, workers=8):
    with ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_make, [(q, frames, held_out) for q in qs]))


def save_checkpoint(path, proposer, meta):
    w = proposer.get_weights()
    m, v, step = proposer.get_state()
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp.npz"
    np.savez(tmp, weights=w, adam_m=m, adam_v=v, step=np.int64(step), meta=np.array(json.dumps(meta)))
    os.replace(tmp, path)


def load_checkpoint(path, proposer, with_state=True):
    with np.load(path, allow_pickle=False) as z:
        proposer.set_weights(z["weights"])
        if with_state:
            proposer.set_state(z["adam_m"], z["adam_v"], int(z["step"]))
        return json.loads(str(z["meta"]))


def load_proposer(path=DEFAULT_WEIGHTS):
    """A proposer with trained weights, or None when there is no checkpoint."""
    import paper_0806_0689_amd as me
    if not os.path.exists(path):
        return None
    p = me.Proposer()
    load_checkpoint(path, p, with_state=False)
    return p


def fs_labels(me, seqs, R):
    """FS motion vectors (device int16 [P, H/16, W/16, 2]) of every pair."""
    out = []
    for s in seqs:
        mv, _, _ = me.fullsearch(s[1:], s[:-1], 16, R)
        out.append(mv)
    return out


def evaluate(me, proposer, seqs, R, fs=True):
    """Mean SAD, NSP and SAD/FS of plain and learned-start DCDS over sequences."""
    import torch
    acc = {"plain_sad": 0.0, "plain_nsp": 0.0, "learned_sad": 0.0, "learned_nsp": 0.0, "fs_sad": 0.0, "blocks": 0}
    for s in seqs:
        cur, ref = s[1:], s[:-1]
        _, ps, pn = me.dcds(cur, ref, 16, R)
        _, ls, ln = me.dcds_learned(proposer, cur, ref, R)
        acc["plain_sad"] += float(ps.double().sum())
        acc["plain_nsp"] += float(pn.double().sum())
        acc["learned_sad"] += float(ls.double().sum())
        acc["learned_nsp"] += float(ln.double().sum())
        if fs:
            _, fsd, _ = me.fullsearch(cur, ref, 16, R)
            acc["fs_sad"] += float(fsd.double().sum())
        acc["blocks"] += ps.numel()
    torch.cuda.synchronize()
    n = acc["blocks"]
    res = {k: acc[k] / n for k in ("plain_sad", "plain_nsp", "learned_sad", "learned_nsp", "fs_sad")}
    res["blocks"] = n
    res["learned_over_plain_sad"] = res["learned_sad"] / res["plain_sad"]
    if fs:
        res["plain_sad_over_fs"] = res["plain_sad"] / res["fs_sad"]
        res["learned_sad_over_fs"] = res["learned_sad"] / res["fs_sad"]
    return res


def train(args):
    import torch
    import paper_0806_0689_amd as me

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    train_np = generate(range(args.sequences), args.frames, workers=args.workers)
    print("generated %d training sequences in %.1f s" % (len(train_np), time.perf_counter() - t0), flush=True)
    seqs = [torch.from_numpy(s).to(dev) for s in train_np]
    del train_np
    labels = fs_labels(me, seqs, args.range)
    torch.cuda.synchronize()
    print("labelled %d pairs with FS +-%d" % (sum(s.shape[0] - 1 for s in seqs), args.range), flush=True)

    p = me.Proposer(seed=args.seed)
    if args.resume and os.path.exists(args.out):
        load_checkpoint(args.out, p)
    rng = np.random.default_rng(args.seed)
    pairs = [(i, t) for i, s in enumerate(seqs) for t in range(s.shape[0] - 1)]
    start_step = p.get_state()[2]
    losses = []
    t0 = time.perf_counter()
    for step in range(start_step, args.steps):
        lr = args.lr * 0.5 * (1.0 + math.cos(math.pi * step / args.steps))
        # One minibatch = args.batch consecutive pairs of one sequence (one call).
        i = int(rng.integers(0, len(seqs)))
        t = int(rng.integers(0, seqs[i].shape[0] - args.batch))
        s = seqs[i]
        loss = p.train_step(s[t + 1:t + 1 + args.batch], s[t:t + args.batch], labels[i][t:t + args.batch], lr)
        if step % args.log_every == 0 or step == args.steps - 1:
            lv = float(loss.cpu()[0])
            losses.append((step, lv))
            print("step %d lr %.2e loss %.4f (%.1f s)" % (step, lr, lv, time.perf_counter() - t0), flush=True)
    torch.cuda.synchronize()
    meta = {"sequences": args.sequences, "frames": args.frames, "range": args.range, "steps": args.steps,
            "batch": args.batch, "lr": args.lr, "seed": args.seed, "losses": losses,
            "train_seconds": time.perf_counter() - t0, "pairs": len(pairs)}
    if args.eval_sequences:
        held = [torch.from_numpy(s).to(dev) for s in
                generate(range(args.eval_sequences), args.frames, held_out=True, workers=args.workers)]
        meta["held_out"] = evaluate(me, p, held, args.range)
        print("held-out:", json.dumps(meta["held_out"]), flush=True)
    save_checkpoint(args.out, p, meta)
    print("saved", args.out, flush=True)
    return meta


def evaluate_checkpoint(args):
    """Held-out evaluation of a saved checkpoint (no training)."""
    import torch
    import paper_0806_0689_amd as me
    dev = torch.device("cuda:0")
    p = load_proposer(args.out)
    if p is None:
        raise SystemExit("no checkpoint at %s" % args.out)
    held = [torch.from_numpy(s).to(dev) for s in
            generate(range(args.eval_sequences), args.frames, held_out=True, workers=args.workers)]
    res = evaluate(me, p, held, args.range)
    print("held-out:", json.dumps(res), flush=True)
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--sequences", type=int, default=40)
    ap.add_argument("--frames", type=int, default=50)
    ap.add_argument("--range", type=int, default=31)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--eval-sequences", type=int, default=4)
    ap.add_argument("--log-every", type=int, default=100)
    ap.add_argument("--resume", action="store_true")
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--eval-only", action="store_true", help="evaluate the checkpoint at --out on held-out data")
    args = ap.parse_args(argv)
    if args.eval_only:
        evaluate_checkpoint(args)
    else:
        train(args)


if __name__ == "__main__":
    main()
