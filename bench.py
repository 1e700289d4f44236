"""Benchmark of the EBIC fitness evaluation on one MI355X.

One step = one evaluation of an 800-individual population (one EBIC
generation's fitness pass) against the resident 436,444 x 64 methylation-
shaped matrix: output initialisation and the evaluation kernel, counts left
on the device. The matrix and the population are resident in HBM before the
timed region starts.

Prints ONE JSON line: the metric (nominal row-trend checks per second, a
check being one (individual, row, column-of-that-individual) triple), the
dominant kernel against its roofline, per-evaluation latency percentiles and
the CPU oracle timed on this host's cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("row-trend checks/sec (pop×rows×cols) at 436,444 rows; % HBM peak; "
          "p50/p99 eval latency")
HBM_PEAK_GBS = 8000.0
# The VALU lane rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12
# 32-bit lane operations per second.
# FP32 / FP16 staging: one 64-lane compare instruction per sub-tile and
# column, counted as 64 compare lane-ops: peak 39.3 T/s.
CMP_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# Byte rank codes: one 32-bit lane op covers four rows, and two column
# steps cost five ops (four v_xad_u32 and one three-input AND): peak
# 4 / 2.5 x 39.3 = 62.9 T row-checks/s.
BYTE_PEAK_TOPS = CMP_PEAK_TOPS * 4 / 2.5
# 16-bit rank codes: the same five ops per two column steps cover two rows
# per lane op: peak 2 / 2.5 x 39.3 = 31.5 T row-checks/s.
HALF_PEAK_TOPS = CMP_PEAK_TOPS * 2 / 2.5
# 10-bit rank codes: three rows per lane op: peak 3 / 2.5 x 39.3 = 47.2 T.
T10_PEAK_TOPS = CMP_PEAK_TOPS * 3 / 2.5
STAGE_BYTES = 3
STAGE_HALVES = 4
STAGE_T10 = 5
STAGE_PAIRS = 6
SWAR_STAGES = (STAGE_BYTES, STAGE_HALVES, STAGE_T10)
# The L2 the pair bitmaps come through: per XCD 16 channels x 128 B per
# clock, eight XCDs at 2.4 GHz: 39.3 TB/s.
L2_PEAK_GBS = 8 * 16 * 128 * 2.4e9 / 1e9
PAIR_CHUNK_ROWS = 2048  # rows of one 32-bit word per lane of a wave
PAIR_WORD_BYTES = 256   # one pair's words on one chunk (64 lanes x 4 B)
ROWS_PER_OP = {STAGE_BYTES: 4, STAGE_HALVES: 2, STAGE_T10: 3}


def alu_roofline(steps, k_ms, staging):
    """The ALU roofline of one launch: `steps` counted by the measurement
    variant (compare instructions, or 64-row sub-tile column steps with byte
    codes) x 64 rows over the kernel time, against the peak of that staging."""
    ach = steps * 64 / (k_ms * 1e-3) / 1e12
    if staging in SWAR_STAGES:
        peak = {STAGE_BYTES: BYTE_PEAK_TOPS, STAGE_HALVES: HALF_PEAK_TOPS, STAGE_T10: T10_PEAK_TOPS}[staging]
        return {"bound": "alu", "achieved": ach, "peak": peak, "unit": "T row-checks/s",
                "frac": ach / peak}
    return {"bound": "alu", "achieved": ach, "peak": CMP_PEAK_TOPS, "unit": "T compare lane-ops/s",
            "frac": ach / CMP_PEAK_TOPS}


def pair_window_pairs(offs, cols, ncols):
    """The distinct ordered column pairs the pair-bitmap kernel reads for
    every chunk: per individual, the pairs of different columns among its
    first eight (after a leading run of repeats of the first column), or
    the one column's diagonal pair."""
    seen = set()
    for i in range(offs.size - 1):
        c = [int(v) for v in cols[offs[i]:offs[i + 1]]]
        if not c or min(c) < 0 or max(c) >= ncols:
            seen.add((0, 0))  # (an invalid individual's header reads pair 0)
            continue
        j = 0
        while j + 1 < len(c) and c[j + 1] == c[0]:
            j += 1
        w = c[j:j + 8]
        w += [w[-1]] * (8 - len(w))
        pairs = {(w[u], w[u + 1]) for u in range(7) if w[u] != w[u + 1]}
        seen |= pairs or {(w[0], w[0])}
    return len(seen)


def pairs_roofline(offs, cols, rows, ncols, steps, k_ms):
    """The HBM roofline of the pair-bitmap kernel: its algorithmic bytes are
    the words of the distinct window pairs on every 2,048-row chunk (each
    read once per launch), the chunks' tie lists, the individuals' headers
    and the counts, over the kernel time."""
    n = offs.size - 1
    chunks = -(-rows // PAIR_CHUNK_ROWS)
    d = pair_window_pairs(offs, cols, ncols)
    nbytes = d * PAIR_WORD_BYTES * chunks + 512 * chunks + 64 * n + 8 * n
    t = k_ms * 1e-3
    ach = nbytes / t / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "algorithmic_bytes": nbytes, "distinct_window_pairs": d, "chunks": chunks,
            "frac_basis": "the bytes this formulation must read per launch (the window pairs' words on every "
                          "chunk); roofline_views.hbm_min_bytes gives the fraction on the method's own minimum, "
                          "the FP32 matrix read once",
            "l2_view": {"bytes": steps * PAIR_WORD_BYTES, "achieved": steps * PAIR_WORD_BYTES / t / 1e9,
                        "peak": L2_PEAK_GBS, "unit": "GB/s",
                        "frac": steps * PAIR_WORD_BYTES / t / 1e9 / L2_PEAK_GBS,
                        "note": "pair-word loads executed (window and tail, counted by the "
                                "measurement variant) x 256 B, against the L2's 16 channels x "
                                "128 B per clock per XCD"}}


def kernel_roofline(stg, steps, k_ms, offs, cols, rows, ncols):
    if stg == STAGE_PAIRS:
        return pairs_roofline(offs, cols, rows, ncols, steps, k_ms)
    return alu_roofline(steps, k_ms, stg)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("ebic_eval.hip", "ebic_chain.inc", "ebic_internal.h", "ebic_pairs.hip", "ebic_prep.h")


def kernel_sources_sha():
    """Digest of the evaluation kernel's sources (the counters in profiles/
    are valid only for the kernel they were taken on)."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1807_09932_amd", "csrc")
    for f in KERNEL_SOURCES:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(launch_units, name="k_eval_methylation_436444x64_traffic.json", shape=None):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel sources changed since the counters were taken, or
    when `shape` (tiles per wave, waves per block, group size, staging) is
    not the launch shape they were taken in."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_sources_sha") != kernel_sources_sha():
        return None
    if shape is None:
        return t.get("hbm_bytes_per_launch")
    want = [int(v) for v in shape]
    for entry in [t] + list(t.get("other_shapes") or []):
        if list(entry.get("launch_shape") or []) == want:
            return entry.get("hbm_bytes_per_launch")
    return None


def cpu_baseline(w, offs, cols, threads, repeats=3):
    import oracle
    rows = w.X.shape[0]
    times = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        oracle.eval_population(w.X, offs, cols, include=False, negative=True, masks=False,
                               threads=threads)
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    checks = rows * int(offs[-1])
    return {"value": checks / dt, "unit": "checks/s", "cores": threads, "kind": "oracle",
            "sample": f"the whole workload: {offs.size - 1} individuals x {rows} rows "
                      f"({checks:.3e} nominal checks) in {dt:.2f} s (median of {repeats})",
            **host_cpu_info()}


def _cpu_model():
    """The processor's full model string (/proc/cpuinfo, else lscpu)."""
    names = []
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                names.append(line.split(":", 1)[1].strip())
    except OSError:
        pass
    name = max(names, key=len) if names else ""
    if len(name) < 12:  # a bare vendor name: ask lscpu
        try:
            import subprocess
            out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
            for line in out.splitlines():
                if line.strip().startswith("Model name"):
                    name = max(name, line.split(":", 1)[1].strip(), key=len)
        except (OSError, subprocess.SubprocessError):
            pass
    return name or "unknown"


def _cgroup_cpus():
    """CPUs the cgroup quota grants this process (cpu.max), or None."""
    try:
        quota, period = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if quota != "max":
            return float(quota) / float(period)
    except (OSError, ValueError):
        pass
    return None


def host_cpu_info():
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count() or 1
    return {"cpu": _cpu_model(), "nproc": affinity, "os_cpu_count": os.cpu_count(),
            "cgroup_cpus": _cgroup_cpus(), "omp_num_threads_env": os.environ.get("OMP_NUM_THREADS")}


def default_cpu_threads():
    """Threads for the oracle baseline: every CPU this process may use (its
    affinity mask), bounded by a cgroup CPU quota when one is set (on a
    shared GPU host the quota is the process's share of the cores)."""
    info = host_cpu_info()
    n = info["nproc"]
    if info["cgroup_cpus"]:
        n = min(n, max(1, int(info["cgroup_cpus"])))
    return max(1, n)


def upload_report(ctx, mat):
    """Resident bytes and upload cost of one matrix (ebic_matrix_get_stats)."""
    st = ctx.stats(mat)
    from paper_1807_09932_amd import ebic
    names = [n for n, b in (("fp32_fill_copy", ebic.SET_FILL_COPY), ("fp16", ebic.SET_FP16),
                            ("fp16_fill", ebic.SET_FP16_FILL), ("u8", ebic.SET_U8),
                            ("u16", ebic.SET_U16), ("u10", ebic.SET_U10), ("pairs", ebic.SET_PAIRS),
                            ("pairs_fill", ebic.SET_PAIRS_FILL)) if st["code_sets"] & b]
    return {"upload_ms": st["upload_ms"], "resident_bytes": st["value_bytes"] + st["code_bytes"],
            "value_bytes": st["value_bytes"], "code_bytes": st["code_bytes"], "code_sets": names,
            "swar_tie_chunks": st["swar_tie_chunks"], "swar_chunks": st["swar_chunks"],
            "upload": "host-to-device copy of the row-major FP32 matrix, layout to column-major, "
                      "rank-code build; host wall clock of ebic_upload_matrix"}


def first_eval_report(ctx, mat, evaluate, X=None, p=None, n=0, **eval_kw):
    """The pair bitmaps are built by the first evaluation that plans them
    (once per matrix and mode): that call's wall time and the bytes it
    added, under the default plan. With X and p, also the first evaluation
    of a second upload of X in the same process (its own bitmaps, built
    again), which holds none of the process's one-time start-up costs."""
    import torch
    before = ctx.stats(mat)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evaluate()
    torch.cuda.synchronize()
    first_ms = (time.perf_counter() - t0) * 1e3
    after = upload_report(ctx, mat)
    rep = {"first_eval_ms": first_ms, "bitmap_bytes": after["code_bytes"] - before["code_bytes"],
           "resident_bytes_after": after["resident_bytes"], "code_sets_after": after["code_sets"],
           "note": "the first evaluation under the default plan: it builds the pairwise order bitmaps "
                   "(every ordered column pair compared once per row, FP32) and then evaluates; later "
                   "evaluations of any population on the matrix reuse them"}
    if X is not None and p is not None:
        m2 = ctx.upload(X)
        try:
            o2 = ctx.outputs(m2, n, masks=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.eval(m2, p, out=o2, **eval_kw)
            torch.cuda.synchronize()
            rep["new_matrix_first_eval_ms"] = (time.perf_counter() - t0) * 1e3
        finally:
            ctx.release(m2)
        rep["new_matrix_note"] = ("the first evaluation on a second upload of the same values in this "
                                  "process: its bitmaps built again, without the process's first-launch "
                                  "costs that first_eval_ms also holds")
    return rep


def roofline_views(executed_steps, k_ms, staging, matrix_bytes, n_ind):
    """The path's two other roofline readings: the HBM roofline of the
    method's minimum traffic (the matrix once, the counts once), and the
    compare-issue rate of the FP32 formulation (two 64-lane compares per
    64-row wave step) against the chip's 32-bit lane rate."""
    t = k_ms * 1e-3
    min_bytes = matrix_bytes + 8 * n_ind
    views = {
        "hbm_min_bytes": {
            "bound": "hbm", "achieved": min_bytes / t / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": min_bytes / t / 1e9 / HBM_PEAK_GBS, "bytes": min_bytes,
            "note": "the method's minimum traffic (the FP32 matrix read once, two int32 counts "
                    "per individual written) over the kernel time; the kernel is bound by "
                    "instruction issue, not by HBM, so this fraction stays small"},
        "fp32_compare_issue": {
            "bound": "alu", "achieved": executed_steps * 2 * 64 / t / 1e12, "peak": CMP_PEAK_TOPS,
            "unit": "T lane-compares/s", "frac": executed_steps * 2 * 64 / t / 1e12 / CMP_PEAK_TOPS,
            "note": "executed 64-row column steps x 2 compares x 64 lanes, as if each step were "
                    "two FP32 compares; above 1 for rank codes, whose one 32-bit lane operation "
                    "compares four (u8), three (u10) or two (u16) rows"},
    }
    if staging == STAGE_PAIRS:
        views["hbm_min_bytes"]["note"] = (
            "the method's minimum traffic (the FP32 matrix read once, two int32 counts per "
            "individual written) over the kernel time; the bitmap kernel reads the words of the "
            "population's window pairs instead (the roofline above), a different byte count: "
            "this fraction is what the same time would give a kernel that read only the matrix")
        # (a pair step ANDs one 32-bit word per lane: 2,048 rows of one
        # column pair, the outcome of 2,048 FP32 compares made at the build)
        views["fp32_compare_issue"] = {
            "bound": "alu", "achieved": executed_steps * PAIR_CHUNK_ROWS / t / 1e12, "peak": CMP_PEAK_TOPS,
            "unit": "T compare outcomes/s",
            "frac": executed_steps * PAIR_CHUNK_ROWS / t / 1e12 / CMP_PEAK_TOPS,
            "note": "executed pair steps x 2,048 rows: the FP32 compare outcomes the kernel "
                    "combines, as if each were a lane compare; above 1 because the bitmaps hold "
                    "32 outcomes per lane word"}
    elif staging not in SWAR_STAGES:
        views["fp32_compare_issue"]["note"] = ("executed 64-row column steps x 2 compares x 64 lanes "
                                               "over the kernel time")
    return views


def _timed(fn, reps, stream):
    """Median wall-clock ms of fn() over reps calls, synchronised each time."""
    import torch
    out = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        stream.synchronize()
        out.append((time.perf_counter() - t0) * 1e3)
    return float(np.median(out))


def bench_batched(ctx, args):
    """64 populations of uneven size (100..1,600 individuals) and skewed
    lengths against one resident 100,000 x 256 matrix: one batched launch
    (a replayed HIP graph) against 64 plain launches, both tuned."""
    import torch
    from paper_1807_09932_amd import ebic, gen
    log("batched: generating 64 populations over a 100,000 x 256 matrix")
    w, pops = gen.batched_100000x256()
    mat = ctx.upload(w.X)
    packed = [gen.csr(p) for p in pops]
    dev = [ctx.population(offsets=o, cols=c) for o, c in packed]
    outs_b = [ctx.outputs(mat, p.n) for p in dev]
    outs_p = [ctx.outputs(mat, p.n) for p in dev]
    reqs = [ctx.request(mat, p, o) for p, o in zip(dev, outs_b)]
    rows = w.X.shape[0]
    checks = sum(gen.nominal_checks(rows, o) for o, _ in packed)
    n_total = sum(p.n for p in dev)
    if args.batch_shape:
        # a forced launch shape (profiling runs: no autotuning launches)
        ctx.set_launch_shape(*[int(x) for x in args.batch_shape.split(",")], 0)
    else:
        log("batched: autotuning plain and batched shapes")
        ctx.set_launch_shape(0, 0, 0, ebic.STAGE_LDS, 0)
        ctx.autotune(reqs)
    stream = torch.cuda.current_stream()

    def batched():
        ctx.eval_batch(reqs)

    def plain():
        for p, o in zip(dev, outs_p):
            ctx.eval(mat, p, out=o)

    batched()
    plain()
    torch.cuda.synchronize()
    same = all(torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
               for a, b in zip(outs_b, outs_p))
    if not same:
        print("bench.py: batched and plain counts differ", file=sys.stderr)
        sys.exit(3)
    # Oracle spot check on two populations.
    import oracle
    for q in (0, len(pops) - 1):
        o, c = packed[q]
        om, on, _, _ = oracle.eval_population(w.X, o, c, negative=True,
                                              threads=default_cpu_threads())
        if not (np.array_equal(outs_b[q][0].cpu().numpy(), om) and
                np.array_equal(outs_b[q][1].cpu().numpy(), on)):
            print("bench.py: batched counts differ from the oracle", file=sys.stderr)
            sys.exit(3)
    for _ in range(3):
        batched()
        plain()
    reps = 20
    b_ms = _timed(batched, reps, stream)
    p_ms = _timed(plain, reps, stream)
    # The batched launch against the compare-issue roofline: executed compare
    # instructions (measurement variant, untimed) over the graph's duration
    # (HIP events around the replay: descriptor copy, prep, evaluation).
    ebic.ebic_set_profiling(ctx.handle, 2)
    batched()
    _, _, b_steps = ebic.ebic_read_profile(ctx.handle)
    ebic.ebic_set_profiling(ctx.handle, 1)
    ebic.ebic_read_profile(ctx.handle)
    for _ in range(reps):
        batched()
    n_l, l_ms, _ = ebic.ebic_read_profile(ctx.handle)
    ebic.ebic_set_profiling(ctx.handle, 0)
    g_ms = l_ms / max(1, n_l)
    bL, bW, bP, b_stg, b_grid = ebic.ebic_plan_batch_shape(ctx.handle, reqs)
    ctx.set_launch_shape()
    upload = upload_report(ctx, mat)
    ctx.release(mat)
    return {
        "workload": "64 populations (%d individuals, lengths 2 + min(38, Exp(mean 5)), "
                    "%.3e nominal checks) over one 100,000 x 256 N(0,1) matrix" % (n_total, checks),
        "batched_ms": b_ms, "plain_ms": p_ms,
        "batched_checks_per_s": checks / (b_ms * 1e-3),
        "plain_checks_per_s": checks / (p_ms * 1e-3),
        "speedup": p_ms / b_ms,
        "equal_results": True,
        "graph_ms": g_ms,
        "executed_compares": b_steps,
        "launch_shape": "L=%d W=%d P=%d stagings=%s blocks=%d" % (bL, bW, bP, sorted(set(b_stg)),
                                                                  b_grid),
        "roofline": batched_roofline(b_steps, g_ms, b_stg, (bL, bW, bP), packed, rows, w.X.shape[1]),
        "timing": "median of %d synchronised calls; batched = one ebic_eval_batch (descriptor "
                  "copy + graph replay), plain = 64 ebic_eval_population calls" % reps,
        "upload": upload,
    }


def batched_roofline(steps, g_ms, stagings, shape, packed, rows, ncols):
    """The batched launch's roofline: on the pair bitmaps, their HBM roofline
    over all populations together (the words of the distinct window pairs
    of every population, once per chunk: the batch walks each chunk for all
    of them); on rank codes, the compare-issue roofline."""
    one = len(set(stagings)) == 1
    if one and stagings[0] == STAGE_PAIRS:
        offs = np.concatenate([[0]] + [o[1:] + sum(int(q[0][-1]) for q in packed[:i])
                                       for i, (o, _) in enumerate(packed)]).astype(np.int64)
        cols = np.concatenate([c[:int(o[-1])] for o, c in packed])
        tr = traffic_from_profile(1, "k_eval_pairs_batch_100000x256_traffic.json", shape + (STAGE_PAIRS,))
        out = {**pairs_roofline(offs, cols, rows, ncols, steps, g_ms), "traffic": tr,
               "time": "the graph replay (descriptor copy, prep, the persistent pairs kernel)"}
        if tr:
            # (each chunk's words of all the batch's pairs, ~16 MB at 256
            # columns, outgrow an XCD's L2: words come in several times)
            out["physical_gbs"] = tr / (g_ms * 1e-3) / 1e9
            out["physical_frac"] = out["physical_gbs"] / HBM_PEAK_GBS
            out["physical_note"] = ("the committed FETCH_SIZE + WRITE_SIZE bytes per launch over the "
                                    "same graph time: L2 fills, from HBM or the Infinity Cache")
        return out
    return {**alu_roofline(steps, g_ms, stagings[0] if one else None),
            "traffic": (traffic_from_profile(1, "k_eval_batch_100000x256_traffic.json", shape + (stagings[0],))
                        if one else None),
            "traffic_note": "HBM bytes per launch of the persistent kernel (committed FETCH_SIZE / "
                            "WRITE_SIZE summary): each staged chunk is read once per group of P "
                            "individuals of each population, mostly from the Infinity Cache"}


def bench_fp32(ctx, args, w, offs, cols):
    """The FP32-tile kernel on the same workload: every row's values staged
    into LDS as FP32 and compared in FP32 (no rank codes), in the best of a
    few launch shapes; its compare instructions against the VALU lane rate."""
    import torch
    from paper_1807_09932_amd import ebic, gen
    rows = w.X.shape[0]
    n = offs.size - 1
    mat = ctx.upload(w.X)
    p = ctx.population(offsets=offs, cols=cols)
    out = ctx.outputs(mat, n)
    stream = torch.cuda.current_stream()
    best = None
    for shape in ((4, 16, 200), (4, 16, 400), (2, 16, 400), (4, 8, 200), (2, 16, 800)):
        ctx.set_launch_shape(*shape, ebic.STAGE_LDS, 0)
        if ebic.ebic_plan_shape(ctx.handle, mat, n)[3] != ebic.STAGE_LDS:
            continue
        ms = _timed(lambda: ctx.eval(mat, p, out=out), 7, stream)
        if best is None or ms < best[1]:
            best = (shape, ms)
    ctx.set_launch_shape(*best[0], ebic.STAGE_LDS, 0)
    L, W, P, stg, blocks = ebic.ebic_plan_shape(ctx.handle, mat, n)
    ctx.eval(mat, p, out=out)
    torch.cuda.synchronize()
    import oracle
    sample = np.arange(0, n, max(1, n // 16))
    so, sc = gen.csr([cols[offs[i]:offs[i + 1]] for i in sample])
    om, on, _, _ = oracle.eval_population(w.X, so, sc, negative=True, threads=default_cpu_threads())
    if not (np.array_equal(out[0].cpu().numpy()[sample], om) and
            np.array_equal(out[1].cpu().numpy()[sample], on)):
        print("bench.py: FP32-tile counts differ from the oracle", file=sys.stderr)
        sys.exit(3)
    ebic.ebic_set_profiling(ctx.handle, 2)
    ctx.eval(mat, p, out=out)
    _, _, steps = ebic.ebic_read_profile(ctx.handle)
    ebic.ebic_set_profiling(ctx.handle, 1)
    ebic.ebic_read_profile(ctx.handle)
    for _ in range(args.steps):
        ctx.eval(mat, p, out=out)
    n_l, ms, _ = ebic.ebic_read_profile(ctx.handle)
    ebic.ebic_set_profiling(ctx.handle, 0)
    ctx.set_launch_shape()
    k_ms = ms / max(1, n_l)
    checks = gen.nominal_checks(rows, offs)
    ctx.release(mat)
    return {"workload": "the same %d x %d matrix and %d individuals" % (rows, w.X.shape[1], n),
            "dtype": "f32",
            "launch_shape": f"best of 5 FP32-tile shapes: L={L} W={W} P={P} staging={stg} blocks={blocks}",
            "kernel_ms": k_ms, "checks_per_s": checks / (k_ms * 1e-3),
            "roofline": alu_roofline(steps, k_ms, stg),
            "ops": "FP32 compares executed per launch: %d wave-wide compare instructions x 64 rows "
                   "(first pair: 3 per 64-row tile, then 1 per column step of each row's oriented "
                   "chain), counted by the measurement variant of the kernel" % steps}


def bench_ea(ctx, args, w=None):
    """The stand-in evolutionary loop around the evaluation on the 436,444 x 64
    matrix: 800 individuals per generation; per generation the host driver
    breeds, the population goes to the device, is evaluated, and its counts
    come back."""
    import torch
    from paper_1807_09932_amd import ebic, gen
    if w is None:
        w, _ = gen.methylation_436444x64()
    rows, ncols = w.X.shape
    mat = ctx.upload(w.X)
    ea = ebic.EA(ncols, 800, 2, 30, seed=180709932)
    gens = 40
    t_host = t_dev = 0.0
    checks = 0
    offs0, cols0, _ = ea.population()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for g in range(gens):
        t1 = time.perf_counter()
        offs, cols, _ = ea.population()
        t2 = time.perf_counter()
        pop = ctx.population(offsets=offs, cols=cols)
        m, _, _, _ = ctx.eval(mat, pop, negative=True)
        counts = m.cpu().numpy()
        t3 = time.perf_counter()
        ea.step(counts)
        t4 = time.perf_counter()
        t_host += (t2 - t1) + (t4 - t3)
        t_dev += t3 - t2
        checks += gen.nominal_checks(rows, offs)
    el = time.perf_counter() - t0
    host_final = ea.population()

    # The same run with breeding on the device (ebic_ea_breed): evaluation
    # and breeding alternate on one stream, the population never leaves the
    # device, and the host waits once at the end.
    def device_run():
        pop = ctx.population(offsets=offs0, cols=cols0)
        m = ctx.outputs(mat, 800, negative=False)[0]
        n, kmax = 800, ea.params.k_max
        bufs = [(torch.empty(n + 1, dtype=torch.int32, device=ctx.device),
                 torch.empty(n * kmax, dtype=torch.int32, device=ctx.device),
                 torch.empty(1, dtype=torch.int32, device=ctx.device)) for _ in range(2)]
        torch.cuda.synchronize()
        t = time.perf_counter()
        for g in range(1, gens + 1):
            ctx.eval(mat, pop, negative=True, out=(m, None, None, None))
            pop, _ = ctx.breed(ea.params, g, pop, m, out=bufs[g & 1])
        torch.cuda.synchronize()
        return time.perf_counter() - t, pop

    device_run()  # (scratch and allocator warm-up)
    el_dev, pop_dev = device_run()
    do = pop_dev.offsets.cpu().numpy()
    same = (np.array_equal(do, host_final[0]) and
            np.array_equal(pop_dev.cols.cpu().numpy()[: int(do[-1])], host_final[1]))
    if not same:
        print("bench.py: the device-bred run differs from the host-bred run", file=sys.stderr)
        sys.exit(3)
    ctx.release(mat)
    ea.close()
    return {"workload": "stand-in evolutionary loop, 800 individuals of 2-30 columns per "
                        "generation, %d x %d matrix, %d generations" % (rows, ncols, gens),
            "generations_per_s": gens / el, "ms_per_generation": el * 1e3 / gens,
            "host_driver_ms_per_generation": t_host * 1e3 / gens,
            "evaluation_ms_per_generation": t_dev * 1e3 / gens,
            "checks_per_s": checks / el,
            "evaluation": "population to the device, ebic_eval_population, matched counts back "
                          "(synchronous)",
            "device_bred": {"ms_per_generation": el_dev * 1e3 / gens,
                            "generations_per_s": gens / el_dev,
                            "checks_per_s": checks / el_dev,
                            "equal_to_host_bred": bool(same),
                            "how": "ebic_eval_population then ebic_ea_breed per generation on one "
                                   "stream, one synchronisation at the end; the final population "
                                   "equals the host-bred run's column for column"}}


def bench_paper_shape(ctx, args):
    """The same evaluation at the paper's dataset width, 436,444 x 310 (a
    541 MB matrix, larger than the Infinity Cache): autotuned, timed, and
    its compares counted."""
    import torch
    from paper_1807_09932_amd import ebic, gen
    log("paper shape: generating 436,444 x 310")
    w, pop = gen.methylation_wide()
    offs, cols = gen.csr(pop)
    rows, ncols = w.X.shape
    mat = ctx.upload(w.X)
    upload = upload_report(ctx, mat)
    p = ctx.population(offsets=offs, cols=cols)
    out = ctx.outputs(mat, p.n)
    ctx.set_launch_shape()
    first_eval = first_eval_report(ctx, mat, lambda: ctx.eval(mat, p, out=out), X=w.X, p=p, n=p.n)
    if args.paper_shape:
        # a forced launch shape (profiling runs: no autotuning launches)
        ctx.set_launch_shape(*[int(x) for x in args.paper_shape.split(",")], 0)
        how = "forced"
    else:
        ctx.set_launch_shape(0, 0, 0, ebic.STAGE_LDS, 0)
        ctx.autotune([ctx.request(mat, p, out)])
        how = "autotuned"
    L, W, P, stg, blocks = ebic.ebic_plan_shape(ctx.handle, mat, p.n, int(offs[-1]))
    ctx.eval(mat, p, out=out)
    torch.cuda.synchronize()
    import oracle
    sample = np.arange(0, p.n, max(1, p.n // 8))
    so, sc = gen.csr([cols[offs[i]:offs[i + 1]] for i in sample])
    om, on, _, _ = oracle.eval_population(w.X, so, sc, negative=True,
                                          threads=default_cpu_threads())
    if not (np.array_equal(out[0].cpu().numpy()[sample], om) and
            np.array_equal(out[1].cpu().numpy()[sample], on)):
        print("bench.py: GPU counts differ from the oracle (paper shape)", file=sys.stderr)
        sys.exit(3)
    ebic.ebic_set_profiling(ctx.handle, 2)
    ctx.eval(mat, p, out=out)
    _, _, steps = ebic.ebic_read_profile(ctx.handle)
    ebic.ebic_set_profiling(ctx.handle, 1)
    ebic.ebic_read_profile(ctx.handle)
    for _ in range(20):
        ctx.eval(mat, p, out=out)
    n_l, ms, _ = ebic.ebic_read_profile(ctx.handle)
    ebic.ebic_set_profiling(ctx.handle, 0)
    k_ms = ms / max(1, n_l)
    checks = gen.nominal_checks(rows, offs)
    ctx.release(mat)
    return {"workload": "%d x %d FP32 Beta(0.5,0.5), 10 planted trends, %d individuals of "
                        "2-30 columns" % (rows, ncols, p.n),
            "upload": upload,
            "first_evaluation": first_eval,
            "roofline_views": roofline_views(steps, k_ms, stg, w.X.nbytes, p.n),
            "launch_shape": f"{how}: L={L} W={W} P={P} staging={stg} blocks={blocks}",
            "kernel_ms": k_ms, "checks_per_s": checks / (k_ms * 1e-3),
            "roofline": {**kernel_roofline(stg, steps, k_ms, offs, cols, rows, ncols),
                         "traffic": traffic_from_profile(1, "k_eval_pairs_methylation_wide_436444x310_traffic.json"
                                                         if stg == STAGE_PAIRS else
                                                         "k_eval_methylation_wide_436444x310_traffic.json",
                                                         (L, W, P, stg))},
            "matrix_once_gbs": w.X.nbytes / (k_ms * 1e-3) / 1e9}


def bench_shard(ctx, args, w, offs, cols):
    """One GPU's share under row sharding across 8 GPUs (Methods, "Support for
    Big Data"): the first slice of ceil(rows/8) rows rounded up to a multiple
    of 64, with the whole population, autotuned and timed; the 8 partial
    counts would then be summed (a 2 x n int32 reduction per generation)."""
    import torch
    from paper_1807_09932_amd import ebic, gen
    rows, ncols = w.X.shape
    per_gpu = -(-rows // 8)
    step = -(-per_gpu // 64) * 64      # slice starts on 64-row mask words
    X = w.X[:step]
    mat = ctx.upload(X)
    p = ctx.population(offsets=offs, cols=cols)
    out = ctx.outputs(mat, p.n)
    ctx.set_launch_shape(0, 0, 0, ebic.STAGE_LDS, 0)
    ctx.autotune([ctx.request(mat, p, out)])
    L, W, P, stg, blocks = ebic.ebic_plan_shape(ctx.handle, mat, p.n, int(offs[-1]))
    ctx.eval(mat, p, out=out)
    torch.cuda.synchronize()
    import oracle
    sample = np.arange(0, p.n, max(1, p.n // 8))
    so, sc = gen.csr([cols[offs[i]:offs[i + 1]] for i in sample])
    om, on, _, _ = oracle.eval_population(X, so, sc, negative=True,
                                          threads=default_cpu_threads())
    if not (np.array_equal(out[0].cpu().numpy()[sample], om) and
            np.array_equal(out[1].cpu().numpy()[sample], on)):
        print("bench.py: GPU counts differ from the oracle (row slice)", file=sys.stderr)
        sys.exit(3)
    ebic.ebic_set_profiling(ctx.handle, 2)
    ctx.eval(mat, p, out=out)
    _, _, steps = ebic.ebic_read_profile(ctx.handle)
    ebic.ebic_set_profiling(ctx.handle, 1)
    ebic.ebic_read_profile(ctx.handle)
    for _ in range(20):
        ctx.eval(mat, p, out=out)
    n_l, ms, _ = ebic.ebic_read_profile(ctx.handle)
    ebic.ebic_set_profiling(ctx.handle, 0)
    k_ms = ms / max(1, n_l)
    checks = gen.nominal_checks(step, offs)
    ctx.release(mat)
    return {"workload": "rows 0-%d of the %d x %d methylation matrix (one of 8 row slices), "
                        "%d individuals" % (step, rows, ncols, p.n),
            "launch_shape": f"L={L} W={W} P={P} staging={stg} blocks={blocks}",
            "kernel_ms": k_ms, "checks_per_s": checks / (k_ms * 1e-3),
            "roofline": kernel_roofline(stg, steps, k_ms, offs, cols, step, ncols)}


def bench_served(ctx, args):
    """Continuous batching of Poisson requests (mean 2,000 req/s) from 16
    EBIC runs over 4 resident matrices; then a closed-loop saturation run and
    the same requests served one plain launch at a time."""
    import torch
    from paper_1807_09932_amd import gen
    from paper_1807_09932_amd.serve import Server
    log("served: uploading 4 matrices, generating request pools")
    ws = gen.served_matrices()
    mats = [ctx.upload(x.X) for x in ws]
    pools = gen.served_pools()
    rows = [x.X.shape[0] for x in ws]
    resident = sum(x.X.nbytes for x in ws)
    budget = 1 << 30
    dur = args.serve_warmup + args.serve_seconds
    reqs = gen.served_requests(dur)
    out = {"workload": "4 resident matrices (10,000 x 100, 50,000 x 200 N(0,1); 200,000 x 64, "
                       "436,444 x 64 Beta(0.5,0.5); %.0f MB); 16 runs, run j on matrix j mod 4; "
                       "populations of 100-800 individuals of 2-30 columns" % (resident / 1e6),
           "hbm_budget_bytes": budget}

    def req_checks(r):
        o, _ = pools[r.matrix][r.pool_index]
        return gen.nominal_checks(rows[r.matrix], o)

    # The load generator is Python: its cyclic garbage collector is paused
    # while it submits, because a collection pause turns scheduled arrivals
    # into bursts that the engine then has to queue (the engine itself runs
    # no Python).
    import gc
    gc.collect()
    gc.disable()
    # Open loop: Poisson arrivals at the scheduled times.
    with Server(ctx, hbm_budget_bytes=budget, slots=4) as srv:
        # warm the graphs / allocator with a few requests first
        for f in [srv.submit(0, mats[m], *pools[m][0]) for m in range(4)]:
            f.result(timeout=60)
        log(f"served: open loop, {len(reqs)} requests over {dur:.1f} s")
        t0 = time.perf_counter()
        futs = []
        reset_done = False
        for r in reqs:
            if not reset_done and r.t_arrival >= args.serve_warmup:
                srv.stats(reset=True)  # the engine's window starts after the warm-up
                reset_done = True
            due = t0 + r.t_arrival
            while True:
                now = time.perf_counter()
                if now >= due:
                    break
                time.sleep(min(2e-4, due - now))
            lag = time.perf_counter() - due
            o, c = pools[r.matrix][r.pool_index]
            futs.append((r, lag, srv.submit(r.run, mats[r.matrix], o, c)))
        lat, done_checks = [], 0
        t_end = 0.0
        for r, lag, f in futs:
            res = f.result(timeout=120)
            if r.t_arrival >= args.serve_warmup:
                lat.append(res.latency_s + lag)
                done_checks += req_checks(r)
        t_end = time.perf_counter() - t0
        st = srv.stats()
    lat = np.array(lat) * 1e3
    out["open_loop"] = {
        "rate_hz": 2000.0, "requests": int(lat.size),
        "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
        "latency": "engine clock: submission to outputs written to the caller's host buffers",
        "client_p50_ms": float(np.percentile(lat, 50)),
        "client_p99_ms": float(np.percentile(lat, 99)),
        "client_max_ms": float(lat.max()),
        "client_latency": "Python load generator (garbage collector paused): scheduled arrival "
                          "to the future's result",
        "served_checks_per_s": done_checks / args.serve_seconds,
        "drain_s_after_last_arrival": max(0.0, t_end - dur),
        "max_ms": st["max_ms"], "queue_p99_ms": st["queue_p99_ms"],
        "batches": st["batches"], "mean_batch": st["mean_batch"],
        "admitted_bytes_high_water": st["admitted_bytes_high_water"],
        "graph_captures_total": st["graph_captures"], "staging_grows": st["staging_grows"],
    }
    log(f"served: open loop p50 {out['open_loop']['p50_ms']:.2f} ms "
        f"p99 {out['open_loop']['p99_ms']:.2f} ms")

    # Closed loop: a fixed number of requests always outstanding.
    seq = reqs[: min(len(reqs), 6000)]
    for depth in (16, 256):
        with Server(ctx, hbm_budget_bytes=budget, slots=4) as srv:
            captures0 = srv.stats()["graph_captures"]
            it = iter(seq)
            pending = []
            done_checks = 0
            t0 = time.perf_counter()
            lat = []
            import concurrent.futures as cf
            live = {}
            for _ in range(depth):
                r = next(it, None)
                if r is None:
                    break
                o, c = pools[r.matrix][r.pool_index]
                live[srv.submit(r.run, mats[r.matrix], o, c)] = r
            # every completed request is replaced at once, so `depth` stay
            # outstanding until the sequence runs out
            while live:
                done, _ = cf.wait(list(live), timeout=120, return_when=cf.FIRST_COMPLETED)
                if not done:
                    raise RuntimeError("closed loop: no request completed within 120 s")
                for f in done:
                    r = live.pop(f)
                    res = f.result()
                    lat.append(res.latency_s)
                    done_checks += req_checks(r)
                    nr = next(it, None)
                    if nr is not None:
                        o, c = pools[nr.matrix][nr.pool_index]
                        live[srv.submit(nr.run, mats[nr.matrix], o, c)] = nr
            el = time.perf_counter() - t0
            st = srv.stats()
        lat = np.array(lat) * 1e3
        out[f"closed_loop_{depth}"] = {
            "outstanding": depth, "requests": len(seq), "checks_per_s": done_checks / el,
            "requests_per_s": len(seq) / el, "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)),
            "latency": "Python client: submission to the future's result (one thread keeps "
                       "`outstanding` requests in flight, replacing each as it completes; one "
                       "thread polls the engine)",
            "engine_p50_ms": st["p50_ms"], "engine_p99_ms": st["p99_ms"],
            "engine_latency": "engine clock: submission to outputs in the caller's host buffers",
            "mean_batch": st["mean_batch"],
            "graph_captures": st["graph_captures"] - captures0,
            "admitted_bytes_high_water": st["admitted_bytes_high_water"]}
        log(f"served: closed loop depth {depth}: {done_checks / el:.3e} checks/s")

    # The same requests, one plain launch each, synchronously.
    seq = reqs[: min(len(reqs), 2000)]
    lat = []
    done_checks = 0
    t0 = time.perf_counter()
    for r in seq:
        t1 = time.perf_counter()
        o, c = pools[r.matrix][r.pool_index]
        p = ctx.population(offsets=o, cols=c)
        m, g, _, _ = ctx.eval(mats[r.matrix], p)
        m.cpu(), g.cpu()
        lat.append(time.perf_counter() - t1)
        done_checks += req_checks(r)
    el = time.perf_counter() - t0
    lat = np.array(lat) * 1e3
    out["plain_per_request"] = {
        "requests": len(seq), "checks_per_s": done_checks / el, "requests_per_s": len(seq) / el,
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "how": "one ebic_eval_population per request, population copied in and counts copied "
               "back synchronously, one request at a time"}
    gc.enable()
    for m in mats:
        ctx.release(m)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--rows", type=int, default=436444, help="(testing only) smaller matrix")
    ap.add_argument("--paper-shape", type=str, default="",
                    help="L,W,P,staging for the 'paper' extra instead of autotuning it")
    ap.add_argument("--batch-shape", type=str, default="",
                    help="L,W,P,staging for the 'batch' extra (both its batched and plain launches) "
                         "instead of autotuning it")
    ap.add_argument("--shape", type=str, default="",
                    help="force the launch shape 'L,W,P[,S]' (64-row tiles per wave, waves per "
                         "block, individuals per group, staging: 0 FP32 tile, 1 direct, "
                         "2 rank codes) instead of autotuning")
    ap.add_argument("--cold-cache-evals", type=int, default=20,
                    help="evaluations timed after streaming a 1 GiB buffer (0 = none)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (3 times), to scale "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE readings to bytes")
    ap.add_argument("--extras", type=str, default="fp32,batch,serve,ea,paper,shard",
                    help="comma list of extra measurements: 'fp32' (the FP32-tile kernel on "
                         "the same workload), 'batch' (64 populations in one "
                         "batched launch vs 64 plain launches), 'serve' (Poisson requests from "
                         "16 runs over 4 resident matrices), 'ea' (the stand-in evolutionary "
                         "loop around the evaluation), 'paper' (436,444 x 310), 'shard' (one of 8 "
                         "row slices of the matrix); '' for none")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-warmup", type=float, default=1.0)
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: the evaluation runs on one GPU; --gpus {args.gpus} is not supported "
              "(sharding rows or populations across GPUs is designed, not built)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1807_09932_amd import ebic, gen

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)

    if args.copy_calibration_mib:
        nbytes = args.copy_calibration_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"bytes_read": nbytes, "bytes_written": nbytes,
                                               "launches": 3}}))
        return

    log("generating the methylation-shaped workload")
    w, pop = gen.methylation_436444x64(rows=args.rows)
    offs, cols = gen.csr(pop)
    rows, ncols = w.X.shape
    n = offs.size - 1
    checks = gen.nominal_checks(rows, offs)

    ctx = ebic.Context(0)
    mat = ctx.upload(w.X)
    upload = upload_report(ctx, mat)
    p = ctx.population(offsets=offs, cols=cols)
    out = ctx.outputs(mat, n, masks=False)
    stream = torch.cuda.current_stream()

    def step():
        ctx.eval(mat, p, include=False, negative=True, masks=False, out=out)

    first_eval = first_eval_report(ctx, mat, step, X=w.X, p=p, n=n, include=False, negative=True, masks=False)
    if args.shape:
        parts = [int(x) for x in args.shape.split(",")]
        L, W, P = parts[:3]
        S = parts[3] if len(parts) > 3 else ebic.STAGE_LDS
        ctx.set_launch_shape(L, W, P, S, 0)
        how = "forced"
    else:
        # The library's autotuner picks the launch shape for this shape class.
        ctx.autotune([ctx.request(mat, p, out, include=False, negative=True)])
        how = "autotuned"
    # The shape the launches take (a forced one may be reduced to what fits).
    L, W, P, stg, blocks = ebic.ebic_plan_shape(ctx.handle, mat, n, int(offs[-1]))
    shape_note = f"{how}: L={L} W={W} P={P} staging={stg} blocks={blocks}"
    log(f"launch shape: {shape_note}")

    # Spot check against the oracle on a sample of individuals.
    import oracle
    sample = np.arange(0, n, max(1, n // 16))
    step()
    torch.cuda.synchronize()
    m_gpu = out[0].cpu().numpy()
    g_gpu = out[1].cpu().numpy()
    so, sc = gen.csr([cols[offs[i]:offs[i + 1]] for i in sample])
    om, on, _, _ = oracle.eval_population(w.X, so, sc, negative=True,
                                          threads=default_cpu_threads())
    if not (np.array_equal(m_gpu[sample], om) and np.array_equal(g_gpu[sample], on)):
        print("bench.py: GPU counts differ from the oracle", file=sys.stderr)
        sys.exit(3)
    log("spot check vs oracle: ok")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # Untimed: executed predicate steps (counting kernel variant).
    ebic.ebic_set_profiling(ctx.handle, 2)
    step()
    _, _, executed_steps = ebic.ebic_read_profile(ctx.handle)
    ebic.ebic_set_profiling(ctx.handle, 0)
    log(f"executed steps per launch: {executed_steps}")

    # Timed region 1 (throughput): K steps back to back with nothing else
    # on the stream, bracketed by synchronisations. An event record costs
    # several microseconds of GPU time per step, so none is taken here.
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # Timed region 2 (the kernel's duration for the roofline): the same K
    # steps with HIP events recorded by the library around every evaluation
    # kernel, on the stream it is launched on.
    ebic.ebic_set_profiling(ctx.handle, 1)
    ebic.ebic_read_profile(ctx.handle)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall_events = time.perf_counter() - t1
    launches, kernel_ms, _ = ebic.ebic_read_profile(ctx.handle)
    ebic.ebic_set_profiling(ctx.handle, 0)
    # Per-step latency: events around each whole step (separate pass).
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    for i in range(args.steps):
        starts[i].record(stream)
        step()
        ends[i].record(stream)
    torch.cuda.synchronize()
    step_ms = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])

    # Cold cache: a 1 GiB buffer is streamed (read and written) before each
    # evaluation, so the matrix comes from HBM rather than the 256 MB
    # Infinity Cache; median kernel time over 20 such evaluations.
    flush = torch.zeros(1 << 28, dtype=torch.float32, device="cuda") if args.cold_cache_evals else None
    cold = []
    for _ in range(args.cold_cache_evals):
        flush.add_(1.0)
        ebic.ebic_set_profiling(ctx.handle, 1)
        step()
        n_c, ms_c, _ = ebic.ebic_read_profile(ctx.handle)
        cold.append(ms_c / max(1, n_c))
    ebic.ebic_set_profiling(ctx.handle, 0)
    del flush
    cold_ms = float(np.median(cold)) if cold else None

    # The measured copy ceiling: a 1 GiB device-to-device copy (read + write).
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(5):
        b.copy_(a)
    c1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * a.numel() * 4 * 5 / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del a, b

    ms_per_step = wall * 1e3 / args.steps
    value = checks / (wall / args.steps)
    k_ms = kernel_ms / max(1, launches)
    roof = kernel_roofline(stg, executed_steps, k_ms, offs, cols, rows, ncols)
    main_traffic = ("k_eval_pairs_methylation_436444x64_traffic.json" if stg == STAGE_PAIRS
                    else "k_eval_methylation_436444x64_traffic.json")

    # End-to-end latency of one generation's evaluation as the host EA sees
    # it: CSR to the device, evaluation, counts back to the host.
    e2e = []
    for i in range(min(50, args.steps)):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pp = ctx.population(offsets=offs, cols=cols)
        ctx.eval(mat, pp, include=False, negative=True, masks=False, out=out)
        _ = out[0].cpu(), out[1].cpu()
        e2e.append(time.perf_counter() - t1)
    e2e = np.array(e2e) * 1e3

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "checks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {STAGE_BYTES: "u8", STAGE_HALVES: "u16", STAGE_T10: "u10", 2: "f16",
                  STAGE_PAIRS: "u1"}.get(stg, "f32"),
        "dtype_note": "the type the evaluation kernel works on: the FP32 compares' outcomes "
                      "as bits (u1: the pairwise order bitmaps, 32 rows per 32-bit lane word, "
                      "combined by AND), the rank codes it stages "
                      "(u8: byte codes, four per 32-bit lane word; u10: 10-bit codes, three per "
                      "word; u16: two per word; f16: FP16 "
                      "codes) or the FP32 values; the resident matrix and the bitmap and code "
                      "builds are FP32 compares, and the counts are exact integers",
        "data": "synthetic",
        "config": {
            "workload": "methylation-shaped plain eval: %d x %d FP32 Beta(0.5,0.5), 10 planted "
                        "trend biclusters, %d individuals of 2-30 columns" % (rows, ncols, n),
            "rows": rows, "cols": ncols, "population": n, "nominal_checks": checks,
            "check": "one (individual, row, column of that individual) triple",
        },
        "roofline": {
            **roof,
            "traffic": traffic_from_profile(1, main_traffic, shape=(L, W, P, stg)),
            "kernel": "k_eval_pairs" if stg == STAGE_PAIRS else "k_eval",
            "launch_shape": shape_note,
            "kernel_ms": k_ms,
            "kernel_ms_cold_cache": cold_ms,
            "timing": "value and ms_per_step: wall clock over the K steps run back to back "
                      "without events; kernel_ms: mean of the HIP event pairs the library "
                      "records around each evaluation kernel on its stream, over a second "
                      "pass of the same K steps (that pass took %.4f ms per step: the events "
                      "cost GPU time)" % (wall_events * 1e3 / args.steps),
            "ops": (("pair bitmaps: per 2,048-row chunk, the words (256 B) of each of the "
                     "population's %d distinct window pairs, read once per launch, plus 512 B of "
                     "tie list per chunk and 72 B per individual (header, counts); %d pair steps "
                     "executed (a wave's AND of one pair word per lane over 2,048 rows, window "
                     "and tail)" % (roof["distinct_window_pairs"], executed_steps))
                    if stg == STAGE_PAIRS else
                    ("row checks executed per launch: %d steps x 64 rows (one step = one column "
                     "of one 64-row sub-tile; the first pair counts one step; early exit per "
                     "chunk of %d lane word(s) per lane), counted by the measurement variant of "
                     "the kernel; peak = 39.3e12 32-bit VALU lane ops/s x %d rows per lane op / "
                     "2.5 ops per column step" % (executed_steps, max(1, L // ROWS_PER_OP.get(stg, 2)),
                                                  ROWS_PER_OP.get(stg, 2)))
                    if stg in SWAR_STAGES else
                    ("FP32 compares executed per launch: %d wave-wide compare instructions x 64 "
                     "rows (first pair: 3 per 64-row tile, then 1 per column step of each row's "
                     "oriented chain; early exit per group of tiles), counted by the measurement "
                     "variant of the kernel" % executed_steps)),
        },
        "roofline_views": roofline_views(executed_steps, k_ms, stg, w.X.nbytes, n),
        "upload": upload,
        "first_evaluation": first_eval,
        "hbm_view": {
            "effective_gbs": 4.0 * checks / (k_ms * 1e-3) / 1e9,
            "effective_frac_of_peak": 4.0 * checks / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "note": "gather-equivalent: 4 B per nominal check; the staged kernel reads the "
                    "matrix once, so this is not physical traffic",
            "matrix_once_gbs": w.X.nbytes / (k_ms * 1e-3) / 1e9,
            "physical_gbs": (traffic_from_profile(1, main_traffic, shape=(L, W, P, stg)) / (k_ms * 1e-3) / 1e9
                             if traffic_from_profile(1, main_traffic, shape=(L, W, P, stg)) else None),
            "copy_ceiling_gbs": copy_gbs,
            "physical_note": "HBM bytes per launch from the committed FETCH_SIZE/WRITE_SIZE "
                             "summary over the measured kernel time; copy ceiling = a 1 GiB "
                             "device copy (bytes read + written per second)",
        },
        "latency_ms": {
            "eval_p50": float(np.percentile(step_ms, 50)),
            "eval_p99": float(np.percentile(step_ms, 99)),
            "eval": "one step (prep and evaluation kernels) between events on the stream, "
                    "a third pass of K steps",
            "end_to_end_p50": float(np.percentile(e2e, 50)),
            "end_to_end_p99": float(np.percentile(e2e, 99)),
            "end_to_end": "CSR host->device, evaluation, counts device->host, synchronous",
        },
    }
    ctx.release(mat)
    extras = {x for x in args.extras.split(",") if x}
    if "fp32" in extras:
        result["fp32_path"] = bench_fp32(ctx, args, w, offs, cols)
    if "batch" in extras:
        result["batched"] = bench_batched(ctx, args)
    if "serve" in extras:
        result["served"] = bench_served(ctx, args)
    if "ea" in extras:
        result["evolutionary_loop"] = bench_ea(ctx, args, w)
    if "paper" in extras:
        result["paper_shape"] = bench_paper_shape(ctx, args)
    if "shard" in extras:
        result["row_shard_of_8"] = bench_shard(ctx, args, w, offs, cols)
    ctx.close()

    if not args.no_cpu_baseline:
        threads = args.cpu_threads or default_cpu_threads()
        log(f"timing the CPU oracle with {threads} threads")
        result["cpu_baseline"] = cpu_baseline(w, offs, cols, threads)
        if threads > 1:
            log("timing the CPU oracle on one thread")
            one = cpu_baseline(w, offs, cols, 1, repeats=1)
            result["cpu_baseline"]["single_thread_value"] = one["value"]
    else:
        result["cpu_baseline"] = None
    print(json.dumps(result))


if __name__ == "__main__":
    main()
