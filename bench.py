"""Benchmark: DCDS motion estimation on 1920x1088 synthetic video, one MI355X.

One step = the whole search over one batch: DCDS (16x16 blocks, range +-15)
over all 59 frame pairs of a 60-frame 1920x1088 uint8 sequence, one library
call (frames resident in HBM before timing starts).  FS, DCDS on 8x8 blocks and
simplified DCDS run over the same frames in their own timed loops and are
reported beside it with their search points, SAD and SAD/FS.

Prints one JSON line.  `value` is DCDS macroblocks per second.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "macroblocks/s at 1080p ±15 (DCDS vs FS vs learned-start), avg SAD pts/MB, SAD/FS"
HBM_PEAK_GBS = 8000.0
W, H, FRAMES, BLOCK, RANGE = 1920, 1088, 60, 16, 15
# Algorithmic HBM bytes per block and launch: the current block and its
# reference block once each, plus 12 bytes of outputs (mv, sad, nsp).
BYTES_PER_BLOCK = lambda b: 2 * b * b + 12  # noqa: E731


def src_digest() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_0806_0689_amd", "csrc")
    for fn in sorted(os.listdir(d)):
        if not fn.startswith("me_"):  # the library's sources only
            continue
        with open(os.path.join(d, fn), "rb") as f:
            h.update(fn.encode() + f.read())
    return h.hexdigest()[:16]


# Before the warmup launches of each timed loop, the launch is repeated for
# this long: an idle GPU starts at lower clocks, and a handful of
# sub-millisecond launches does not bring it to its steady state (measured:
# the headline launch reads about 10% slower after 5 warmup launches alone).
SETTLE_MS = 200.0


def time_launches(fn, steps, warmup, torch):
    """Per-launch durations (ms) from HIP events on the launch stream, after
    SETTLE_MS of untimed repeats and `warmup` untimed launches."""
    t_end = time.perf_counter() + SETTLE_MS * 1e-3
    while time.perf_counter() < t_end:
        for _ in range(8):
            fn()
        torch.cuda.synchronize()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        starts[i].record()
        fn()
        ends[i].record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    per = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    return wall / steps, sum(per) / len(per), per


def valu_rates():
    """VALU issue rates of the SAD instructions on this device, from the
    calibration program that build() compiles (run as a child process)."""
    import subprocess
    exe = os.path.join(ROOT, "paper_0806_0689_amd", "valu_rates")
    if not os.path.exists(exe):
        return {"status": "calibration program not built"}
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    if r.returncode != 0:
        return {"status": "calibration program failed: %s" % r.stderr[-300:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def counters_for(kernel: str):
    """The rocprofv3 counter record of a kernel (HBM bytes and VALU
    instructions per launch), if it was taken on this source."""
    p = os.path.join(ROOT, "profiles", "traffic_%s.json" % kernel)
    if not os.path.exists(p):
        return None
    with open(p) as f:
        rec = json.load(f)
    if rec.get("src_digest") != src_digest():
        return None
    return rec


def traffic_for(kernel: str):
    """HBM bytes per launch measured by rocprofv3 counters, if taken on this source."""
    rec = counters_for(kernel)
    return rec.get("bytes_per_launch") if rec else None


# VALU issue peak: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD every 4
# cycles, at the 2.4 GHz peak clock.
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4


def valu_issue_for(kernel: str, ms: float):
    """The kernel's VALU instruction count per launch (from its counter
    record) over this run's launch time, against the issue peak."""
    rec = counters_for(kernel)
    if not rec or "valu_insts_per_launch" not in rec:
        return None
    rate = rec["valu_insts_per_launch"] / (ms * 1e-3)
    return {"insts_per_launch": rec["valu_insts_per_launch"], "achieved": rate, "peak": VALU_ISSUE_PEAK,
            "unit": "wave64 instructions/s", "frac": rate / VALU_ISSUE_PEAK,
            "lanes_active": rec.get("lanes_active"), "source": rec.get("summary")}


def fs_roofline(rates, achieved):
    """Full search against the v_qsad_pk_u16_u8 issue peak.  The calibration
    times the instructions in seconds and converts at 2.4 GHz; a plain
    integer add (v_xad_u32) issues every 4 cycles per SIMD, so its reading
    gives the clock the calibration actually ran at.  The peak is stated at
    the 2.4 GHz peak clock: the qsad cost in true cycles (its reading times
    4 / the add's), at 256 CUs x 4 SIMDs x 2.4 GHz, 1024 absolute differences
    per wave instruction."""
    cyc = rates["cycles_per_wave_instruction"]
    measured_peak = rates["absdiff_per_s"]["v_qsad_pk_u16_u8"]
    clock = 2.4 * 4.0 / cyc["v_xad_u32"]
    qsad_cycles = cyc["v_qsad_pk_u16_u8"] * 4.0 / cyc["v_xad_u32"]
    peak = rates["cus"] * 4 * 2.4e9 / qsad_cycles * 64 * 16
    return {"achieved_absdiff_per_s": achieved, "peak_absdiff_per_s": peak, "frac": achieved / peak,
            "peak_clock_ghz": 2.4, "qsad_cycles_per_wave_instruction": qsad_cycles,
            "calibration_clock_ghz": clock, "peak_at_measured_clock": measured_peak,
            "frac_at_measured_clock": achieved / measured_peak}


_CPU_SEQ = None  # the sequence the forked oracle workers read


def _oracle_pairs(pairs):
    import oracle
    for p in pairs:
        oracle.dcds(_CPU_SEQ[p + 1], _CPU_SEQ[p], BLOCK, RANGE)
    return len(pairs) * (W // BLOCK) * (H // BLOCK)


def _oracle_fs_pair(p):
    import oracle
    oracle.fullsearch(_CPU_SEQ[p + 1], _CPU_SEQ[p], BLOCK, RANGE)
    return (W // BLOCK) * (H // BLOCK)


def host_info():
    """The host's logical CPU count, the CPUs this process may use, and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "cpu_model": model}


def cpu_baseline(seq, budget_s=6.0):
    """The CPU oracle as written (gcc -O2 scalar C) on the same workload: one
    thread, then one process per host core (at most 16, the host share of one
    GPU) over the frame pairs.  Runs before the GPU is touched, so the worker
    processes are plain forks."""
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    import oracle
    global _CPU_SEQ
    _CPU_SEQ = seq
    oracle.lib()
    pairs = list(range(FRAMES - 1))
    n1, t0, reps1 = 0, time.perf_counter(), 0
    while time.perf_counter() - t0 < budget_s:
        n1 += _oracle_pairs(pairs)
        reps1 += 1
    dt1 = time.perf_counter() - t0
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    chunks = [pairs[i::cores] for i in range(cores)]
    with ProcessPoolExecutor(max_workers=cores, mp_context=multiprocessing.get_context("fork")) as ex:
        list(ex.map(_oracle_pairs, [[0]] * cores))  # start the workers
        nk, t0, repsk = 0, time.perf_counter(), 0
        while time.perf_counter() - t0 < budget_s:
            nk += sum(ex.map(_oracle_pairs, chunks))
            repsk += 1
        dtk = time.perf_counter() - t0
    res = {"value": nk / dtk, "unit": "MB/s", "cores": cores, "kind": "oracle",
           "sample": "DCDS over all %d pairs of the same 1920x1088 sequence, %d passes (%.1f s), gcc -O2 scalar C, "
                     "one process per core over the pairs" % (FRAMES - 1, repsk, dtk),
           "single_core_value": n1 / dt1,
           "single_core_sample": "%d passes (%.1f s), one thread" % (reps1, dt1)}
    t0 = time.perf_counter()
    oracle.fullsearch(seq[1], seq[0], BLOCK, RANGE)
    fs_dt = time.perf_counter() - t0
    res["fs_single_core_value"] = (W // BLOCK) * (H // BLOCK) / fs_dt
    res["fs_sample"] = "FS on pair 0 only, one thread (%.1f s)" % fs_dt
    # FS on every core at once: one pair per process (pairs 0 .. cores-1).
    with ProcessPoolExecutor(max_workers=cores, mp_context=multiprocessing.get_context("fork")) as ex:
        list(ex.map(_oracle_pairs, [[0]] * cores))  # start the workers
        t0 = time.perf_counter()
        nf = sum(ex.map(_oracle_fs_pair, range(cores)))
        fsk_dt = time.perf_counter() - t0
    res["fs_all_core_value"] = nf / fsk_dt
    res["fs_all_core_sample"] = "FS on pairs 0..%d, one pair per process on %d cores (%.1f s)" % (
        cores - 1, cores, fsk_dt)
    res["host"] = host_info()
    res["compiler"] = "gcc %s" % " ".join(oracle.CC_FLAGS)
    print("# cpu oracle: %.3g MB/s on %d cores, %.3g MB/s on one" % (res["value"], cores, res["single_core_value"]),
          file=sys.stderr, flush=True)
    return res


def batch_leg(me, torch, dev, args):
    """64 streams (16 each of 176x144, 352x288, 1280x720, 1920x1088), 30 frames,
    16x16 blocks, +-15.  The autotuner first picks the kernel layout on this
    batch; then every timed launch takes a different job table (the stream
    list rotated by 16 per launch, so the sizes at each table position change
    from launch to launch) through the same captured graph, against one
    me_dcds call per stream."""
    from synth import batch_streams
    t0 = time.perf_counter()
    seqs = [torch.from_numpy(s).to(dev) for s in batch_streams(64, 30)]
    print("# generated 64 streams in %.1f s" % (time.perf_counter() - t0), file=sys.stderr, flush=True)
    pairs = [(s[1:], s[:-1]) for s in seqs]
    blocks = sum((s.shape[0] - 1) * (s.shape[1] // 16) * (s.shape[2] // 16) for s in seqs)
    cfg, tune_ms = me.autotune(pairs, 16, RANGE, me.ME_ALGO_DCDS, reps=3)
    tables = []
    for k in range(4):
        order = [(i + 16 * k) % 64 for i in range(64)]
        tables.append(me.make_jobs([pairs[i] for i in order], 16))
    stream = torch.cuda.current_stream().cuda_stream
    turn = [0]

    def launch():
        jobs = tables[turn[0] % 4][0]
        turn[0] += 1
        rc = me.me_batch(jobs, 64, me.ME_ALGO_DCDS, 16, RANGE, stream)
        assert rc == 0, rc

    single = [me.dcds(c, r, 16, RANGE) for (c, r) in pairs]  # the per-stream calls' own outputs

    def per_stream():
        for (c, r), o in zip(pairs, single):
            me.dcds(c, r, 16, RANGE, out=o)

    steps = max(4, min(args.steps, 20))
    _, ms_batch, _ = time_launches(launch, steps, args.warmup, torch)
    _, ms_loop, _ = time_launches(per_stream, steps, args.warmup, torch)
    # Every table's outputs, written by its last launch, against the
    # per-stream calls, element by element.
    for k in range(4):
        launch_k = tables[k][0]
        assert me.me_batch(launch_k, 64, me.ME_ALGO_DCDS, 16, RANGE, stream) == 0
    torch.cuda.synchronize()
    for k in range(4):
        for i, o in enumerate(tables[k][1]):
            ref_o = single[(i + 16 * k) % 64]
            if not all(torch.equal(x, y) for x, y in zip(o, ref_o)):
                raise AssertionError("batch table %d job %d differs from its per-stream call" % (k, i))
    me.me_set_config(16, RANGE, None)  # the other legs keep the built-in layout
    nsp = sum(float(o[2].double().sum()) for o in tables[0][1]) / blocks
    res = {"streams": 64, "frames": 30, "blocks_per_launch": blocks, "ms_per_launch": ms_batch,
           "checked": "all 4 tables x 64 jobs equal to the per-stream calls, element by element",
           "mb_per_s": blocks / (ms_batch * 1e-3), "per_stream_calls_ms": ms_loop,
           "per_stream_calls_mb_per_s": blocks / (ms_loop * 1e-3), "nsp_mean": nsp,
           "tables": "4 rotations of the stream list, one per launch",
           "config": {"rows_per_lane": cfg[0], "waves_per_group": cfg[1], "tiles_per_grab": cfg[2],
                      "source": "me_autotune",
                      "autotune_ms": tune_ms}}
    print("# batch: %.4f ms per launch (%.3g MB/s), autotuned %s; 64 separate calls %.4f ms" % (
        ms_batch, res["mb_per_s"], cfg, ms_loop), file=sys.stderr, flush=True)
    return res


def learned_leg(me, torch, cur, ref, R, steps, warmup, fs_sad=None, plain=None):
    """Learned-start DCDS (proposer inference + seeded DCDS, timed together)."""
    from paper_0806_0689_amd.train import DEFAULT_WEIGHTS, load_proposer
    p = load_proposer()
    if p is None:
        return {"status": "no trained checkpoint at %s" % DEFAULT_WEIGHTS}
    fn = lambda: me.dcds_learned(p, cur, ref, R)  # noqa: E731
    mv, sad, nsp = fn()
    _, ms, _ = time_launches(fn, steps, warmup, torch)
    _, ms_cnn, _ = time_launches(lambda: p.infer(cur, ref, R), steps, warmup, torch)
    blocks = sad.numel()
    res = {"mb_per_s": blocks / (ms * 1e-3), "ms_per_step": ms, "proposer_ms": ms_cnn,
           "nsp_mean": float(nsp.double().mean()), "sad_mean": float(sad.double().mean())}
    if fs_sad:
        res["sad_over_fs"] = res["sad_mean"] / fs_sad
    if plain:
        res["sad_over_plain_dcds"] = res["sad_mean"] / plain["sad_mean"]
        res["nsp_over_plain_dcds"] = res["nsp_mean"] / plain["nsp_mean"]
    print("# learned: %.4f ms/step (proposer %.4f ms), %.3g MB/s, nsp %.3f, sad %.1f" % (
        ms, ms_cnn, res["mb_per_s"], res["nsp_mean"], res["sad_mean"]), file=sys.stderr, flush=True)
    return res


def quality_leg(me, torch, cur, ref, R, steps, warmup):
    """The measures of §IV for FS, DCDS and DCDS^S on the headline workload
    (FS vectors as the truth), and the cost of the fused squared-error
    epilogue and of the per-pair summary kernel."""
    import numpy as np
    P, H, W = cur.shape
    out = {}
    runs = {}
    for name, algo in (("fs", me.ME_ALGO_FS), ("dcds", me.ME_ALGO_DCDS), ("dcds_s", me.ME_ALGO_DCDS_S)):
        runs[name] = me.search(cur, ref, 16, R, algo, sse=True)
    truth = runs["fs"][0]
    for name, (mv, sad, nsp, sse) in runs.items():
        rec = me.frame_quality(mv, sad, sse, truth, block=16)
        nb = float(rec["blocks"].sum())
        out[name] = {
            "mad": float(rec["sad"].sum()) / (nb * 256), "mse": float(rec["sse"].sum()) / (nb * 256),
            "psnr_db": float(np.mean(rec["psnr"])), "distance": float(rec["dist"].sum()) / nb,
            "probability": float(rec["equal"].sum()) / nb, "nsp": float(nsp.double().mean()),
        }
    fn = lambda: me.search(cur, ref, 16, R, me.ME_ALGO_DCDS, sse=True)  # noqa: E731
    fn()
    _, ms_sse, _ = time_launches(fn, steps, warmup, torch)
    mv, sad, nsp, sse = runs["dcds"]
    buf = torch.empty(P * me.QUALITY_BYTES, dtype=torch.uint8, device=cur.device)
    st = torch.cuda.current_stream().cuda_stream
    qf = lambda: me.me_frame_quality(mv.data_ptr(), sad.data_ptr(), sse.data_ptr(), truth.data_ptr(),  # noqa: E731
                                     W, H, P, 16, buf.data_ptr(), st)
    qf()
    _, ms_q, _ = time_launches(qf, steps, warmup, torch)
    out["dcds_with_sse_ms"] = ms_sse
    out["summary_kernel_ms"] = ms_q
    print("# quality: dcds+sse %.4f ms, summary %.4f ms; psnr fs %.3f dcds %.3f dcds_s %.3f dB; "
          "dcds distance %.4f probability %.4f" % (
              ms_sse, ms_q, out["fs"]["psnr_db"], out["dcds"]["psnr_db"], out["dcds_s"]["psnr_db"],
              out["dcds"]["distance"], out["dcds"]["probability"]), file=sys.stderr, flush=True)
    return out


def mvp_leg(me, torch, cur, ref, steps, warmup):
    """The MVP statistics of §II-C over the headline sequence in the paper's
    +-7 window: time of one full pass (full search with the statistics
    epilogue over all pairs, then the tables), and the synthetic data's
    distribution beside the paper's Table III / Fig. 3 figures."""
    R = 7
    n = 2 * R + 1
    counts = (torch.zeros(n * n, dtype=torch.int32, device=cur.device),
              torch.zeros((9, n * n), dtype=torch.int32, device=cur.device),
              torch.zeros((n * n, 25), dtype=torch.int32, device=cur.device))

    def one():
        for c in counts:
            c.zero_()
        me.mvp_stats(cur, ref, 16, R, counts=counts)

    one()
    _, ms, _ = time_launches(one, max(3, min(steps, 10)), warmup, torch)
    t = me.mvp_tables(counts, R)
    out = {
        "ms_per_pass": ms,
        "p00": float(t["quarter"][0, 0]),
        "bx": [float(v) for v in t["bx"][R - 2:R + 3]], "by": [float(v) for v in t["by"][R - 2:R + 3]],
        "ax_var": float(sum(t["ax"][i] * (i - R) ** 2 for i in range(n))),
        "ay_var": float(sum(t["ay"][i] * (i - R) ** 2 for i in range(n))),
        "regions": [float(v) for v in t["regions"]], "eta": [float(v) for v in t["eta"]],
        "paper": {"p00": 0.5805, "bx": [0.0151, 0.0718, 0.5805, 0.0562, 0.0440],
                  "by": [0.0031, 0.0295, 0.5805, 0.0277, 0.0035]},
    }
    print("# mvp: %.4f ms per pass; P(0,0) %.4f; var x %.3f y %.3f; eta %s" % (
        ms, out["p00"], out["ax_var"], out["ay_var"], [round(v, 4) for v in out["eta"]]), file=sys.stderr, flush=True)
    return out


def e2e_leg(me, torch, seq_np, dev, args):
    """The headline call end to end from host memory: the 60 frames copied
    from pinned host memory to the GPU, the DCDS call, and its outputs copied
    back, timed by the host clock around a synchronised step (the PCIe-
    inclusive rate; the headline times the call on resident frames)."""
    host = torch.from_numpy(seq_np).pin_memory()
    seq = torch.empty(host.shape, dtype=torch.uint8, device=dev)
    P, Hc, Wc = host.shape[0] - 1, host.shape[1], host.shape[2]
    outs = [torch.empty((P, Hc // 16, Wc // 16, 2), dtype=torch.int16).pin_memory(),
            torch.empty((P, Hc // 16, Wc // 16), dtype=torch.int32).pin_memory(),
            torch.empty((P, Hc // 16, Wc // 16), dtype=torch.int32).pin_memory()]

    def step():
        seq.copy_(host, non_blocking=True)
        res = me.dcds(seq[1:], seq[:-1], 16, RANGE)
        for o, r in zip(outs, res):
            o.copy_(r, non_blocking=True)
        torch.cuda.synchronize()

    for _ in range(3):
        step()
    n = max(5, min(args.steps, 20))
    t0 = time.perf_counter()
    for _ in range(n):
        step()
    ms = (time.perf_counter() - t0) * 1e3 / n
    blocks = P * (Hc // 16) * (Wc // 16)
    res = {"ms_per_step": ms, "mb_per_s": blocks / (ms * 1e-3), "bytes_h2d": int(host.numel()),
           "bytes_d2h": sum(int(o.numel() * o.element_size()) for o in outs),
           "what": "pinned host frames -> HBM, me_dcds over 59 pairs, outputs -> pinned host; host clock"}
    print("# e2e: %.4f ms per step from host memory (%.3g MB/s)" % (ms, res["mb_per_s"]), file=sys.stderr,
          flush=True)
    return res


def small_config_leg(me, torch, dev, k, args):
    """Configs 1 (176x144, one pair), 2 (352x288, 300 frames, 299 pairs) and 6
    (352x288, 60 frames, the paper's operating point), 16x16 blocks, +-7: FS,
    plain DCDS and learned-start DCDS, one launch per step over every pair of
    the sequence.  Beside the §IV measures it reports how often DCDS finds the
    FS vector (Table IX's probability, with FS as the truth) and how often FS
    finds (0, 0) (Table II's centre probability)."""
    from synth import make_config
    seq_np = make_config(k)
    seq = torch.from_numpy(seq_np).to(dev)
    cur, ref = seq[1:], seq[:-1]
    R = 7
    steps = max(5, min(args.steps, 50))
    P, Hc, Wc = cur.shape
    blocks = P * (Hc // 16) * (Wc // 16)
    out = {"workload": "%dx%d uint8, %d frames (%d pairs), 16x16, +-%d, %d blocks per step" % (
        Wc, Hc, P + 1, P, R, blocks)}
    mvs = {}
    for name, fn in (("fs", lambda: me.fullsearch(cur, ref, 16, R)), ("dcds", lambda: me.dcds(cur, ref, 16, R))):
        mvs[name], sad, nsp = fn()
        _, ms, _ = time_launches(fn, steps, args.warmup, torch)
        out[name] = {"mb_per_s": blocks / (ms * 1e-3), "ms_per_step": ms, "sad_mean": float(sad.double().mean()),
                     "nsp_mean": float(nsp.double().mean())}
    out["dcds"]["sad_over_fs"] = out["dcds"]["sad_mean"] / out["fs"]["sad_mean"]
    out["dcds"]["p_fs_vector"] = float((mvs["dcds"] == mvs["fs"]).all(-1).double().mean())
    out["fs"]["p_zero_vector"] = float((mvs["fs"] == 0).all(-1).double().mean())
    out["dcds_learned"] = learned_leg(me, torch, cur, ref, R, steps, args.warmup, out["fs"]["sad_mean"],
                                      out["dcds"])
    print("# config%d: fs %.4f ms (%.3g MB/s), dcds %.4f ms (%.3g MB/s), sad/fs %.4f, nsp %.3f, "
          "P(dcds = fs) %.3f, P(fs = 0) %.3f" % (
              k, out["fs"]["ms_per_step"], out["fs"]["mb_per_s"], out["dcds"]["ms_per_step"], out["dcds"]["mb_per_s"],
              out["dcds"]["sad_over_fs"], out["dcds"]["nsp_mean"], out["dcds"]["p_fs_vector"],
              out["fs"]["p_zero_vector"]), file=sys.stderr, flush=True)
    return out


def config5_leg(me, torch, dev, args):
    """3840x2160, 60 frames, +-31, 16x16: plain DCDS, learned-start DCDS and FS."""
    from synth import make_config
    t0 = time.perf_counter()
    seq = torch.from_numpy(make_config(5)).to(dev)
    print("# generated 3840x2160 x 60 in %.1f s" % (time.perf_counter() - t0), file=sys.stderr, flush=True)
    cur, ref = seq[1:], seq[:-1]
    steps = max(3, min(args.steps, 10))
    out = {"workload": "3840x2160 uint8, 60 frames (59 pairs), 16x16, +-31"}
    fn = lambda: me.fullsearch(cur, ref, 16, 31)  # noqa: E731
    _, fs_sad, fs_nsp = fn()
    _, ms_fs, _ = time_launches(fn, 3, 1, torch)
    blocks = fs_sad.numel()
    out["fs"] = {"mb_per_s": blocks / (ms_fs * 1e-3), "ms_per_step": ms_fs, "sad_mean": float(fs_sad.double().mean()),
                 "nsp_mean": float(fs_nsp.double().mean())}
    fn = lambda: me.dcds(cur, ref, 16, 31)  # noqa: E731
    _, sad, nsp = fn()
    _, ms, _ = time_launches(fn, steps, args.warmup, torch)
    out["dcds"] = {"mb_per_s": blocks / (ms * 1e-3), "ms_per_step": ms, "sad_mean": float(sad.double().mean()),
                   "nsp_mean": float(nsp.double().mean())}
    out["dcds"]["sad_over_fs"] = out["dcds"]["sad_mean"] / out["fs"]["sad_mean"]
    out["dcds_learned"] = learned_leg(me, torch, cur, ref, 31, steps, args.warmup, out["fs"]["sad_mean"],
                                      out["dcds"])
    print("# config5: fs %.3f ms, dcds %.4f ms" % (ms_fs, ms), file=sys.stderr, flush=True)
    return out


def main():
    global SETTLE_MS
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--only", default="",
                    help="comma list of extra legs to run (fs,dcds8,fs8,dcds_s,learned,batch,quality,mvp,e2e,"
                         "config1,config2,config6,4k); "
                         "dcds always runs")
    ap.add_argument("--sweep", action="store_true",
                    help="time every DCDS kernel configuration (rows per lane x waves per group) and exit")
    ap.add_argument("--sweep-range", type=int, default=RANGE, help="search range of --sweep")
    ap.add_argument("--settle-ms", type=float, default=SETTLE_MS,
                    help="untimed repeats of each timed launch before its warmup, in ms (0: none)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first copy 256 MiB device-to-device (a known-size kernel for counter calibration)")
    args = ap.parse_args()
    SETTLE_MS = args.settle_ms
    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path "
              "(blocks are independent; sharding across GPUs needs no exchange).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_0806_0689_amd as me
    from synth import make_config

    t0 = time.perf_counter()
    seq_np = make_config(3)
    print("# generated %s in %.1f s" % (seq_np.shape, time.perf_counter() - t0), file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu and not args.sweep:
        cpu = cpu_baseline(seq_np)  # before the GPU is initialised (forked workers)
    dev = torch.device("cuda:0")
    seq = torch.from_numpy(seq_np).to(dev)
    cur, ref = seq[1:], seq[:-1]
    P = FRAMES - 1
    legs = set(args.only.split(",")) if args.only else {"dcds", "fs", "dcds8", "fs8", "dcds_s", "learned", "batch",
                                                          "quality", "mvp", "e2e", "config1", "config2", "config6",
                                                          "4k"}
    if args.calib_copy:
        src = torch.ones(256 << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)                 # runtime copy kernel: reads and writes 256 MiB
        torch.add(src, 1, out=dst)     # elementwise kernel: reads and writes 256 MiB
        torch.cuda.synchronize()
        del src, dst

    if args.sweep:
        SR = args.sweep_range
        for B, rpls in ((16, (1, 2, 4)), (8, (1, 2))):
            for rpl in rpls:
                for wpg in (1, 2, 4, 8):
                    if me.me_set_config(B, SR, (rpl, wpg)) != me.ME_OK:
                        continue
                    fn = lambda: me.dcds(cur, ref, B, SR)  # noqa: E731
                    try:
                        fn()
                    except me.MEError as e:  # a window too large for LDS
                        print(json.dumps({"block": B, "rows_per_lane": rpl, "waves_per_group": wpg,
                                          "range": SR, "error": str(e)}), flush=True)
                        continue
                    _, ms, _ = time_launches(fn, args.steps, args.warmup, torch)
                    nb = P * (H // B) * (W // B)
                    print(json.dumps({"block": B, "rows_per_lane": rpl, "waves_per_group": wpg, "range": SR,
                                      "ms": ms, "mb_per_s": nb / (ms * 1e-3)}), flush=True)
            me.me_set_config(B, SR, None)
        return

    results = {}

    def leg(name, fn, steps, blocks_per_step):
        outs = fn()
        torch.cuda.synchronize()
        ms_wall, ms_ev, per = time_launches(fn, steps, args.warmup, torch)
        mv, sad, nsp = outs
        results[name] = {
            "mb_per_s": blocks_per_step / (ms_ev * 1e-3),
            "ms_per_step": ms_ev,
            "ms_per_step_wall": ms_wall,
            "nsp_mean": float(nsp.double().mean()),
            "sad_mean": float(sad.double().mean()),
            "_sad": sad,
        }
        print("# %s: %.4f ms/step (events), %.4f ms wall, %.3g MB/s, nsp %.3f, sad %.1f" % (
            name, ms_ev, ms_wall, results[name]["mb_per_s"], results[name]["nsp_mean"],
            results[name]["sad_mean"]), file=sys.stderr, flush=True)

    blocks16 = P * (H // 16) * (W // 16)
    blocks8 = P * (H // 8) * (W // 8)
    leg("dcds", lambda: me.dcds(cur, ref, 16, RANGE), args.steps, blocks16)
    if "fs" in legs:
        leg("fs", lambda: me.fullsearch(cur, ref, 16, RANGE), max(3, min(args.steps, 10)), blocks16)
        # FS is bound by v_qsad_pk_u16_u8 issue (16 absolute differences per
        # lane and instruction); its peak is measured, not assumed.
        rates = valu_rates()
        fs = results["fs"]
        fs["valu_roofline"] = {"bound": "alu", "instr": "v_qsad_pk_u16_u8", "rates": rates}
        if "absdiff_per_s" in rates:
            fs["valu_roofline"].update(fs_roofline(rates, fs["nsp_mean"] * 256 * blocks16 / (fs["ms_per_step"] * 1e-3)))
            r = fs["valu_roofline"]
            print("# fs: %.3g absolute differences/s, %.0f%% of the v_qsad_pk_u16_u8 peak at 2.4 GHz (%.3g), "
                  "%.0f%% of the rate measured at the calibration's clock (%.2f GHz)" % (
                      r["achieved_absdiff_per_s"], 100 * r["frac"], r["peak_absdiff_per_s"],
                      100 * r["frac_at_measured_clock"], r["calibration_clock_ghz"]), file=sys.stderr, flush=True)
    if "dcds8" in legs:
        leg("dcds8", lambda: me.dcds(cur, ref, 8, RANGE), args.steps, blocks8)
    if "fs8" in legs:
        leg("fs8", lambda: me.fullsearch(cur, ref, 8, RANGE), max(3, min(args.steps, 10)), blocks8)
        if "dcds8" in results:
            results["dcds8"]["sad_over_fs"] = results["dcds8"]["sad_mean"] / results["fs8"]["sad_mean"]
    if "dcds_s" in legs:
        leg("dcds_s", lambda: me.dcds(cur, ref, 16, RANGE, algo=me.ME_ALGO_DCDS_S), args.steps, blocks16)
    if "learned" in legs:
        fs_mean = results["fs"]["sad_mean"] if "fs" in results else None
        results["dcds_learned"] = learned_leg(me, torch, cur, ref, RANGE, args.steps, args.warmup, fs_mean,
                                              results["dcds"])
    if "batch" in legs:
        results["batch"] = batch_leg(me, torch, dev, args)
    extra = {}
    if "quality" in legs:
        extra["quality"] = quality_leg(me, torch, cur, ref, RANGE, args.steps, args.warmup)
    if "mvp" in legs:
        extra["mvp_stats_r7"] = mvp_leg(me, torch, cur, ref, args.steps, args.warmup)
    if "e2e" in legs:
        extra["end_to_end"] = e2e_leg(me, torch, seq_np, dev, args)
    for k in (1, 2, 6):
        if "config%d" % k in legs:
            extra["config%d" % k] = small_config_leg(me, torch, dev, k, args)
    if "4k" in legs:
        del seq, cur, ref
        extra["config_4k_r31"] = config5_leg(me, torch, dev, args)
    if "fs" in legs:
        fs_sad = results["fs"]["sad_mean"]
        for k in ("dcds", "dcds_s"):
            if k in results:
                results[k]["sad_over_fs"] = results[k]["sad_mean"] / fs_sad
    for r in results.values():
        r.pop("_sad", None)

    d = results["dcds"]
    bytes_launch = BYTES_PER_BLOCK(16) * blocks16
    achieved = bytes_launch / (d["ms_per_step"] * 1e-3) / 1e9
    traffic = traffic_for("k_dcds_1080p")
    valu = valu_issue_for("k_dcds_1080p", d["ms_per_step"])
    line = {
        "metric": METRIC,
        "value": d["mb_per_s"],
        "unit": "MB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "settle_ms": SETTLE_MS,
        "ms_per_step": d["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {
            "workload": "DCDS, 1920x1088 uint8 luma, 60 frames (59 pairs, one launch), 16x16 blocks, range +-15",
            "frames": FRAMES, "pairs": P, "block": 16, "range": RANGE, "blocks_per_step": blocks16,
            "generator": "synth config 3, seed 3",
        },
        "algos": results,
        **extra,
        "roofline": {
            "kernel": "k_dcds<16,%d,%d,15>" % me.me_get_config(16, RANGE)[:2],
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "bytes_per_block": BYTES_PER_BLOCK(16),
            "traffic": traffic,
            # HBM bytes the counters measured, over this run's launch time.
            "traffic_gbs": traffic / (d["ms_per_step"] * 1e-3) / 1e9 if traffic else None,
            "traffic_frac": traffic / (d["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS if traffic else None,
            # What limits the kernel in practice: its VALU issue rate (the
            # larger fraction of the two).
            "valu_issue": valu,
            "limiter": ("valu_issue" if valu and valu["frac"] > achieved / HBM_PEAK_GBS else "hbm"),
        },
        "cpu_baseline": None,
    }
    line["cpu_baseline"] = cpu
    print(json.dumps(line))


if __name__ == "__main__":
    main()
