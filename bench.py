#!/usr/bin/env python3
"""Throughput of batched segmented NCC on one MI355X.

A step is one pass of the whole hot path over one batch held in HBM: sum
tables of every frame, FP32-compensated scoring of every (frame, template)
pair at every offset with top-k selection, and FP64 re-scoring of the
candidates' neighbourhoods with the fine approximation (one graph launch).

Default workload ("coarse-fine"): 256 frames 1280x720 x 32 templates with
sides U{24..96}, coarse sigma_max 16 (top-32 per pair), fine sigma_max 4 on
+-2 px neighbourhoods.  `--workload batched` runs 16 frames 1920x1080 x 64
templates (sides U{16..192}, sigma_max U{4,8,12,16}, top-5) instead;
`--workload threshold` runs the paper's own two-threshold search (Section 5)
on 4 frames 1920x1080 x 4 templates 64x64 with relative thresholds (value =
fast plus slow evaluations per second); `--workload prep` times the host
template preparation alone (1024 templates, both approximations);
`--workload large` runs one 3840x2160 frame with a 640x480 and a 384x384
template (areas beyond one exact f^2 box; the first in the direct form),
top-5 per pair.

Prints one JSON line.  value = coarse offset x segment evaluations per
second of the whole step.
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

METRIC = "offset×segment evals/sec + frames/sec, batched FP32 vs plain FP64, |Δρ|≤1e-5"
UNIT = "offset×segment evals/s"

# VALU lane operations of the method per offset x segment evaluation: 3 integer
# add/sub for the box sum (Eq. (11)), 1 integer multiply-add for the mean term
# of Eq. (12), 1 int->float conversion, 1 FMA with c_i, 3 add/sub of the
# compensated sum.
OPS_PER_EVAL = 9
# 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz: non-packed VALU lane operations/s
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# LDS read bandwidth measured on MI355X with paper_2502_01286_amd/lds_probe
# (profiles/lds_read_bandwidth.txt), bytes/clock/CU at 2.4 GHz x 256 CUs: the
# widest read form (ds_read_b128) is the peak; ds_read2st64_b32, the form the
# scoring kernel's corner reads use, is reported beside it.  16 bytes (4
# corners) per eval by the method's definition.
LDS_B128_B_PER_CLK = 171.7
LDS_READ2ST64_B_PER_CLK = 102.7
LDS_PEAK_TBS = LDS_B128_B_PER_CLK * 256 * 2.4e9 / 1e12
LDS_READ2ST64_TBS = LDS_READ2ST64_B_PER_CLK * 256 * 2.4e9 / 1e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("tile_kernel.hpp", "device_util.hpp", "tile_entry.hip", "sncc_internal.hpp")


def kernel_source_hash():
    """First 16 hex digits of the SHA-256 over the scoring kernel's sources."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2502_01286_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload):
    """HBM bytes of the scoring stage (its launches of tile_kernel) from the
    committed rocprofv3 --pmc summary (FETCH_SIZE and WRITE_SIZE, each scaled
    by what the counter reads for a copy kernel of known size), or None when
    it was taken on another kernel source.  The summary is text: `key: value`
    lines, `#` comments."""
    path = os.path.join(ROOT, "profiles", f"tile_kernel_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    d = {}
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#") and ":" in line:
                key, val = line.split(":", 1)
                d[key.strip()] = val.strip()
    if d.get("kernel_sources_sha256_16") != kernel_source_hash():
        return None
    try:
        return int(d.get("scoring_stage_bytes", d["bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def make_workload(name):
    from workloads import synth
    if name == "coarse-fine":
        return synth.coarse_fine_256x32()
    if name == "large":
        return synth.large_3840x2160()
    if name == "batched":
        return synth.batch_16x64()
    if name == "coarse-fine-small":
        return synth.coarse_fine_256x32(n_frames=16, n_templates=8)
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(wl, coarse_segs_k, budget_s=15.0, max_pairs=1024, gpu_topk=None,
                 gpu_best=None):
    """The oracle (NumPy FP64), as it stands, on a seeded sample of pairs of
    the same workload, one pair per worker process.  With the GPU's results
    of the same step (top-k lists, and final matches when refining), an
    untimed second pass compares them with the oracle on those pairs."""
    import numpy as np
    from concurrent.futures import ProcessPoolExecutor
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    rng = np.random.default_rng(12345)
    order = rng.permutation(len(wl.pairs))
    # bound the sample: estimated cost ~ offsets x K per pair
    est = lambda p: (wl.M - wl.templates[wl.pairs[p][1]].shape[1] + 1) * \
        (wl.N - wl.templates[wl.pairs[p][1]].shape[0] + 1) * coarse_segs_k[wl.pairs[p][1]]
    chosen, work = [], 0.0
    rate_guess = 1.4e8 * cores         # evals/s of the NumPy oracle (rough, for sizing only)
    for p in order:
        if len(chosen) >= max_pairs or work / rate_guess > budget_s:
            break
        chosen.append(int(p))
        work += est(p)
    jobs = [(wl.frames[wl.pairs[p][0]], wl.templates[wl.pairs[p][1]], wl.sigmas[wl.pairs[p][1]],
             wl.fine_sigma, wl.k) for p in chosen]
    # template preparation happens before timing, as in the paper's split
    with ProcessPoolExecutor(max_workers=cores) as ex:
        preps = list(ex.map(_cpu_prep, jobs))
        t0 = time.perf_counter()
        res = list(ex.map(_cpu_pair, jobs, preps))
        dt = time.perf_counter() - t0
        evals = sum(r[0] for r in res)
        parity = None
        if gpu_topk is not None:
            checks = list(ex.map(_cpu_check, jobs, preps, [r[1:] for r in res],
                                 [gpu_topk[p] for p in chosen],
                                 [gpu_best[p] if gpu_best is not None else None for p in chosen]))
            parity = _summarise_checks(checks, wl.k)
    out = {"value": evals / dt, "unit": UNIT, "cores": cores, "kind": "oracle",
           "cpu_model": _cpu_model(),
           "sample": f"{len(chosen)} seeded (frame, template) pairs of the same workload: "
                     f"full coarse rho map (FP64) + top-{wl.k}"
                     + (" + FP64 fine re-score of the +-2 px neighbourhoods" if wl.fine_sigma else "")
                     + f", {dt:.1f} s wall on {cores} processes"}
    return out, parity


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_prep(job):
    import oracle as O
    f, t, sc, sf, k = job
    c = O.precompute_template_approximation(t, sc)
    fi = O.precompute_template_approximation(t, sf) if sf else None
    return c, fi


def _cpu_pair(job, prep):
    """Timed oracle work of one pair: the whole coarse map, its top-k (and the
    next entry, for the set gap) and, when refining, the coarse-fine result."""
    import numpy as np
    import oracle as O
    f, t, sc, sf, k = job
    c, fi = prep
    tables = O.sum_tables(f)
    N, M = f.shape
    cmap = O.rho_map(f, c, tables=tables)
    best = None
    if fi is not None:
        res = O.coarse_fine(*tables, c, fi, M, N, k=k, radius=2, coarse_map=cmap)
        ref, best = list(res["coarse"]), res["best"]
    else:
        ref = O.topk(cmap, k)
    # the value of rank k + 1 (for the set gap only; a partial sort, a few ms)
    flat = cmap.ravel()
    if flat.size > k:
        ref.append((-1, -1, float(np.partition(flat, flat.size - k - 1)[flat.size - k - 1])))
    return cmap.size * c.K, ref, best


SET_GAP = 2e-5      # rank-k / rank-k+1 oracle gap that fixes the top-k set (2 x 1e-5)


def _cpu_check(job, prep, oracle_res, g_topk, g_best):
    """Untimed: the GPU's results of one pair against the oracle.  Coarse:
    rho at every reported offset, and the set of offsets where the oracle's
    rank-k / rank-k+1 gap exceeds SET_GAP.  Final (refining workloads): the
    oracle's fine step over the GPU's own candidates (Section 5, steps 7f-i),
    which equals the oracle's whole coarse-fine result when the candidate set
    is fixed; its argmax must be the GPU's wherever its fine top-2 margin
    exceeds 1e-9."""
    import numpy as np
    import oracle as O
    from oracle import select as OSEL
    f, t, sc, sf, k = job
    c, fi = prep
    ref, cf_best = oracle_res
    tables = O.sum_tables(f)
    N, M = f.shape
    nu, nv = M - c.W + 1, N - c.H + 1
    u = np.array([m[0] for m in g_topk], np.int64)
    v = np.array([m[1] for m in g_topk], np.int64)
    r = np.array([m[2] for m in g_topk], np.float64)
    ok = u >= 0
    want = O.rho_at(*tables, c, u[ok], v[ok])
    d = {"coarse_err": float(np.abs(want - r[ok]).max()) if ok.any() else 0.0,
         "set_fixed": False, "set_equal": None}
    gap = ref[k - 1][2] - ref[k][2] if len(ref) > k else np.inf
    if gap > SET_GAP:
        d["set_fixed"] = True
        d["set_equal"] = {(int(a), int(b)) for a, b in zip(u[ok], v[ok])} == \
            {(a, b) for a, b, _ in ref[:k]}
    if g_best is not None and fi is not None:
        cands = [(int(a), int(b), 0.0) for a, b in zip(u[ok], v[ok])]
        cu, cv = OSEL.neighbourhood(cands, 2, nu, nv)
        fr = O.rho_at(*tables, fi, cu, cv)
        order = np.lexsort((cu, cv, -fr))
        i0 = order[0]
        margin = fr[i0] - fr[order[1]] if len(order) > 1 else np.inf
        bu, bv, br = int(g_best[0]), int(g_best[1]), float(g_best[2])
        d["fine_err"] = abs(br - float(O.rho_at(*tables, fi, bu, bv)))
        d["final_decided"] = bool(margin > 1e-9)
        d["final_match"] = (bu, bv) == (int(cu[i0]), int(cv[i0])) if margin > 1e-9 else \
            br >= fr[i0] - 1e-9
        if d["set_fixed"] and d["set_equal"]:
            d["final_vs_oracle_cf"] = (bu, bv) == tuple(cf_best[:2]) or margin <= 1e-9
    return d


def _summarise_checks(checks, k):
    out = {"pairs": len(checks),
           "coarse_max_abs_drho": max(c["coarse_err"] for c in checks),
           "topk_sets_fixed": sum(c["set_fixed"] for c in checks),
           "topk_sets_equal": sum(bool(c["set_equal"]) for c in checks if c["set_fixed"]),
           "k": k, "set_gap": SET_GAP, "tolerance": 1e-5}
    if checks and "fine_err" in checks[0]:
        out.update({
            "fine_max_abs_drho": max(c["fine_err"] for c in checks),
            "final_argmax_checked": len(checks),
            "final_argmax_match": sum(bool(c["final_match"]) for c in checks),
            "final_decided_by_margin_1e-9": sum(c["final_decided"] for c in checks),
            "final_vs_oracle_coarse_fine": sum(bool(c.get("final_vs_oracle_cf")) for c in checks),
            "fine_tolerance": 1e-9})
    return out


# ------------------------------------------------ the two-threshold search
PRECISION = 0.9           # Section 5's precision
OPS_PER_SLOW_EVAL = 5     # 3 integer add/sub (Eq. (11)), 1 int->FP64 convert, 1 FP64 FMA
FP64_VALU_PEAK_TOPS = VALU_PEAK_TOPS   # FP64 vector FMA issues at the FP32 lane rate


def _cpu_threshold_prep(job):
    import oracle as O
    f, t = job
    sf, ss = O.paper_sigmas(t)
    return O.precompute_template_approximation(t, sf), O.precompute_template_approximation(t, ss)


def _cpu_threshold_pair(job, prep, max_slow):
    import numpy as np
    import oracle as O
    f, t = job
    fa, sl = prep
    N, M = f.shape
    s, s2 = O.sum_tables(f)
    fmap = O.rho_map(f, fa, tables=(s, s2))
    thr_f = PRECISION * fa.rho_max
    cv, cu = np.nonzero(fmap >= thr_f)
    cu, cv = cu[:max_slow], cv[:max_slow]
    r = O.rho_at(s, s2, sl, cu, cv)
    int((r >= PRECISION * sl.rho_max).sum())
    return fmap.size * fa.K + len(cu) * sl.K


def cpu_threshold_baseline(wl, budget_s=15.0):
    """The oracle's threshold_match steps on one pair per process: the whole
    fast map, then the slow rho at the first survivors (bounded)."""
    from concurrent.futures import ProcessPoolExecutor
    cores = max(1, min(16, len(os.sched_getaffinity(0)), len(wl.pairs)))
    jobs = [(wl.frames[b], wl.templates[t]) for b, t in wl.pairs[:cores]]
    max_slow = int(2e6 * budget_s / 15.0)
    with ProcessPoolExecutor(max_workers=cores) as ex:
        preps = list(ex.map(_cpu_threshold_prep, jobs))
        t0 = time.perf_counter()
        evals = sum(ex.map(_cpu_threshold_pair, jobs, preps, [max_slow] * len(jobs)))
        dt = time.perf_counter() - t0
    return {"value": evals / dt, "unit": UNIT, "cores": cores, "kind": "oracle",
            "sample": f"{len(jobs)} (frame, template) pairs of the same workload, one per "
                      f"process: whole fast rho map (FP64) + slow rho at up to {max_slow} "
                      f"survivors each, {dt:.1f} s wall"}


def run_threshold(args):
    import numpy as np
    import torch
    import paper_2502_01286_amd as S
    from workloads import synth

    wl = synth.threshold_4x4()
    B, N, M = len(wl.frames), wl.N, wl.M
    log(f"[bench] threshold search: {B} frames {M}x{N}, {len(wl.templates)} templates "
        f"{wl.templates[0].shape[1]}x{wl.templates[0].shape[0]}, {len(wl.pairs)} pairs")
    t0 = time.perf_counter()
    fast_l, slow_l, tf, ts, Kf, Ks = [], [], [], [], [], []
    for t in wl.templates:
        sigma_t = float(np.asarray(t, np.float64).std())     # population deviation
        a, _, rf = S.sncc_segment_template(t, 0.99 * sigma_t)
        b, _, rs = S.sncc_segment_template(t, 0.1 * sigma_t)
        fast_l.append(a)
        slow_l.append(b)
        tf.append(PRECISION * rf)
        ts.append(PRECISION * rs)
        Kf.append(len(a))
        Ks.append(len(b))
    prep_ms = (time.perf_counter() - t0) * 1e3
    log(f"[bench] prep {prep_ms:.1f} ms, K fast {Kf}, K slow {Ks}")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ctx = S.sncc_ctx_create(0)
    Ws = [t.shape[1] for t in wl.templates]
    Hs = [t.shape[0] for t in wl.templates]
    fast = S.sncc_upload_templates(ctx, fast_l, Ws, Hs)
    slow = S.sncc_upload_templates(ctx, slow_l, Ws, Hs)
    f = torch.from_numpy(np.stack(wl.frames)).to(dev)
    P = S.sncc_sat_pitch(M)
    s = torch.empty((B, N + 1, P), dtype=torch.int32, device=dev)
    s2 = torch.empty_like(s)
    offs = [(M - Ws[t] + 1) * (N - Hs[t] + 1) for _, t in wl.pairs]
    cap = sum(offs)
    cand = torch.empty((cap, 6), dtype=torch.int32, device=dev)
    out = torch.empty((cap, 6), dtype=torch.int32, device=dev)
    counts = torch.zeros(4, dtype=torch.int32, device=dev)

    def step():
        S.sncc_build_sats(ctx, f, s, s2)
        S.sncc_threshold_match(ctx, fast, slow, tf, ts, s, s2, B, M, N, wl.pairs, cand, out,
                               counts)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    # stage times from separate steps: reading them waits for each step
    S.sncc_ctx_set_timing(ctx, True)
    stage = []
    for _ in range(max(3, min(args.steps, 10))):
        step()
        stage.append(S.sncc_ctx_stage_ms(ctx))
    S.sncc_ctx_set_timing(ctx, False)
    n_cand, n_out = (int(x) for x in counts[:2].cpu())
    hits = S.decode_hits(cand, n_cand)
    per_pair = np.bincount(hits["pair"], minlength=len(wl.pairs))
    fast_evals = int(sum(o * Kf[t] for o, (_, t) in zip(offs, wl.pairs)))
    slow_evals = int(sum(int(c) * Ks[t] for c, (_, t) in zip(per_pair, wl.pairs)))
    ms_fast = float(np.median([x[0] for x in stage]))
    ms_slow = float(np.median([x[1] for x in stage]))
    value = (fast_evals + slow_evals) / (ms_per_step / 1e3)
    log(f"[bench] {args.steps} steps: {ms_per_step:.3f} ms/step (fast {ms_fast:.3f} ms, slow "
        f"{ms_slow:.3f} ms); {n_cand} survivors, {n_out} matches")
    fast_tops = OPS_PER_EVAL * fast_evals / (ms_fast / 1e3) / 1e12
    slow_tops = OPS_PER_SLOW_EVAL * slow_evals / (ms_slow / 1e3) / 1e12
    if ms_slow >= ms_fast:
        roof = {"bound": "alu", "achieved": round(slow_tops, 3),
                "peak": round(FP64_VALU_PEAK_TOPS, 2), "unit": "TOP/s (FP64 VALU lane ops)",
                "frac": round(slow_tops / FP64_VALU_PEAK_TOPS, 4), "traffic": None,
                "kernel": "slow_kernel (FP64 slow pass)", "kernel_ms": round(ms_slow, 4),
                "ops_per_eval": OPS_PER_SLOW_EVAL, "evals_per_launch": slow_evals}
    else:
        roof = {"bound": "alu", "achieved": round(fast_tops, 3), "peak": round(VALU_PEAK_TOPS, 2),
                "unit": "TOP/s (VALU lane ops)", "frac": round(fast_tops / VALU_PEAK_TOPS, 4),
                "traffic": None, "kernel": "tile_kernel (compacting sink)",
                "kernel_ms": round(ms_fast, 4), "ops_per_eval": OPS_PER_EVAL,
                "evals_per_launch": fast_evals}
    roof["stages"] = {"fast_ms": round(ms_fast, 4), "fast_tops": round(fast_tops, 3),
                      "slow_ms": round(ms_slow, 4), "slow_tops": round(slow_tops, 3)}
    cpu = None
    if not args.no_cpu:
        log("[bench] CPU oracle baseline")
        cpu = cpu_threshold_baseline(wl, budget_s=args.cpu_budget)
        log(f"[bench] cpu {cpu}")
    S.sncc_tmpl_destroy(fast)
    S.sncc_tmpl_destroy(slow)
    S.sncc_ctx_destroy(ctx)
    line = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "threshold", "frames": B, "width": M, "height": N,
                   "templates": len(wl.templates), "pairs": len(wl.pairs),
                   "precision": PRECISION, "sigma_fast": "0.99 sigma_t",
                   "sigma_slow": "0.1 sigma_t", "K_fast": Kf, "K_slow": Ks,
                   "fast_evals": fast_evals, "slow_evals": slow_evals,
                   "survivors": n_cand, "matches": n_out,
                   "arith": "u32 box sums, f32 compensated fast rho, f64 slow rho"},
        "frames_per_s": B / (ms_per_step / 1e3), "prep_ms_host": prep_ms,
        "roofline": roof, "plain_fp64": None, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


# --------------------------------------------- batched template preparation
def _cpu_prep_sample(job):
    import oracle as O
    t, sf, ss = job
    O.precompute_template_approximation(t, sf)
    O.precompute_template_approximation(t, ss)
    return 1


def run_prep(args):
    """Template preparation (Section 5, lines 1-5 of the algorithm, the part the
    paper times separately): both approximations of many templates on host
    threads.  Host only; no device work."""
    import numpy as np
    import paper_2502_01286_amd as S
    from workloads import synth

    wl = synth.prep_1024()
    ts = wl.templates
    sd = [float(np.asarray(t, np.float64).std()) for t in ts]
    sig = [0.99 * x for x in sd] + [0.1 * x for x in sd]
    both = ts + ts
    log(f"[bench] preparation: {len(ts)} templates (sides {min(t.shape[0] for t in ts)}.."
        f"{max(t.shape[0] for t in ts)}), fast and slow approximations")
    for _ in range(args.warmup):
        S.sncc_segment_templates(both, sig, 5000, 0)
    times = []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        lists, su, rm, st = S.sncc_segment_templates(both, sig, 5000, 0)
        times.append(time.perf_counter() - t0)
    t_all = float(np.median(times))
    t0 = time.perf_counter()
    S.sncc_segment_templates(both, sig, 5000, 1)
    t_one = time.perf_counter() - t0
    threads = os.cpu_count() or 1
    K = [len(a) for a in lists]
    log(f"[bench] {t_all * 1e3:.1f} ms on all threads, {t_one * 1e3:.1f} ms on one; K fast "
        f"{min(K[:len(ts)])}..{max(K[:len(ts)])}, K slow {min(K[len(ts):])}..{max(K[len(ts):])}")
    cpu = None
    if not args.no_cpu:
        from concurrent.futures import ProcessPoolExecutor
        cores = max(1, min(16, len(os.sched_getaffinity(0))))
        rng = np.random.default_rng(4242)
        pick = rng.permutation(len(ts))
        jobs = [(ts[i], 0.99 * sd[i], 0.1 * sd[i]) for i in pick]
        done, t0 = 0, time.perf_counter()
        with ProcessPoolExecutor(max_workers=cores) as ex:
            for chunk in range(0, len(jobs), cores * 4):
                done += sum(ex.map(_cpu_prep_sample, jobs[chunk:chunk + cores * 4]))
                if time.perf_counter() - t0 > args.cpu_budget:
                    break
        dt = time.perf_counter() - t0
        cpu = {"value": done / dt, "unit": "templates/s", "cores": cores, "kind": "oracle",
               "sample": f"{done} seeded templates of the same set, both approximations, "
                         f"{dt:.1f} s wall on {cores} processes"}
        log(f"[bench] cpu {cpu}")
    line = {
        "metric": "template preparation (both approximations per template)",
        "value": len(ts) / t_all, "unit": "templates/s", "n_gpus": 0,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_all * 1e3,
        "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic",
        "config": {"workload": "prep", "templates": len(ts), "host_threads": threads,
                   "sigma_fast": "0.99 sigma_t", "sigma_slow": "0.1 sigma_t", "K_max": 5000,
                   "K_fast": [min(K[:len(ts)]), max(K[:len(ts)])],
                   "K_slow": [min(K[len(ts):]), max(K[len(ts):])],
                   "one_thread_templates_per_s": len(ts) / t_one},
        "roofline": None, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


# ------------------------------------------- per-configuration measurements
def _band_map(job):
    """Oracle map of offset rows [v0, v1) of one frame (the map of image rows
    [v0, v1 + H - 1)), in sub-bands of 16 rows that keep NumPy's arrays in
    cache; box sums are the same integers from any table origin."""
    import numpy as np
    import oracle as O
    rows, ta, nvb = job
    out = np.empty((nvb, rows.shape[1] - ta.W + 1))
    for a in range(0, nvb, 16):
        b = min(nvb, a + 16)
        out[a:b] = O.rho_map(rows[a:b + ta.H - 1], ta)
    return out


def _oracle_map(ex, n_proc, f, ta):
    import numpy as np
    nv = f.shape[0] - ta.H + 1
    step = max(16, -(-nv // (4 * n_proc)))
    jobs = [(np.ascontiguousarray(f[v0:min(nv, v0 + step) + ta.H - 1]), ta, min(nv, v0 + step) - v0)
            for v0 in range(0, nv, step)]
    return np.concatenate(list(ex.map(_band_map, jobs)), axis=0)


def _events_ms(torch, fn, reps):
    """Mean time per call of back-to-back calls between two events: at least
    `reps` calls, more for short calls (about 2 ms in all, at most 200), so
    that a call of a few microseconds is timed in steady state."""
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    fn()
    e1.record()
    torch.cuda.synchronize()
    reps = max(reps, min(200, int(2.0 / max(e0.elapsed_time(e1), 1e-3))))
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _single_config(S, torch, ctx, ex, n_proc, wl, sigma, k_max, full_oracle, reps=5):
    """One frame, one template: device times of the sum tables, the FP32
    map, the FP32 top-1 (batched persistent form) and the plain FP64 map;
    FP32 and FP64 against the oracle (whole map, or a seeded sample of
    offsets plus the neighbourhoods of both sides' best offsets)."""
    import numpy as np
    import oracle as O
    f, t = wl.frames[0], wl.templates[0]
    N, M = f.shape
    H, W = t.shape
    segs, su, _ = S.sncc_segment_template(t, sigma, k_max)
    K = len(segs)
    tm = S.sncc_upload_templates(ctx, [segs], [W], [H])
    d = torch.from_numpy(f).cuda().unsqueeze(0)
    P = S.sncc_sat_pitch(M)
    s = torch.empty((1, N + 1, P), dtype=torch.int32, device="cuda")
    s2 = torch.empty_like(s)
    nu, nv = M - W + 1, N - H + 1
    r32 = torch.empty((nv, nu), dtype=torch.float32, device="cuda")
    r64 = torch.empty((nv, nu), dtype=torch.float64, device="cuda")
    top1 = torch.zeros((1, 1, 3), dtype=torch.int32, device="cuda")
    ms_sat = _events_ms(torch, lambda: S.sncc_build_sats(ctx, d, s, s2), reps)
    ms32 = _events_ms(torch, lambda: S.sncc_score(ctx, tm, 0, s, s2, M, N, S.SNCC_FP32_KAHAN,
                                                  r32), reps)
    ms_top1 = _events_ms(torch, lambda: S.sncc_argmax(ctx, tm, s, s2, 1, M, N, [(0, 0)],
                                                      S.SNCC_FP32_KAHAN, top1), reps)
    ms64 = _events_ms(torch, lambda: S.sncc_score(ctx, tm, 0, s, s2, M, N, S.SNCC_FP64, r64),
                      max(2, reps // 2))
    # from the frame: tile-local sum tables (when the template allows) and the
    # global form (tables of the frame, then the map)
    rf = torch.empty((nv, nu), dtype=torch.float32, device="cuda")
    fr = d[0]
    forms = {}
    for name, form in (("tile_local", S.SNCC_FORM_TILE_LOCAL), ("global", S.SNCC_FORM_GLOBAL)):
        try:
            forms[name] = round(_events_ms(torch, lambda: S.sncc_score_frame(
                ctx, tm, 0, fr, rf, form=form), reps), 4)
        except S.SnccError:
            forms[name] = None
    forms["auto_picks"] = "tile_local" if S.sncc_score_frame(ctx, tm, 0, fr, rf) == \
        S.SNCC_FORM_TILE_LOCAL else "global"
    g32 = r32.cpu().numpy().astype(np.float64)
    g64 = r64.cpu().numpy()
    b1 = S.decode_matches(top1)[0, 0]
    S.sncc_tmpl_destroy(tm)
    evals = nu * nv * K
    ta = O.precompute_template_approximation(t, sigma, k_max)
    a32 = np.unravel_index(int(np.argmax(g32)), g32.shape)[::-1]
    a64 = np.unravel_index(int(np.argmax(g64)), g64.shape)[::-1]
    out = {"frame": f"{M}x{N}", "template": f"{W}x{H}", "sigma": sigma,
           "K_max": k_max if k_max < 10 ** 8 else None, "sigma_used": su, "K": K,
           "offsets": nu * nv, "evals": evals,
           "ms_sat": round(ms_sat, 4), "ms_fp32_map": round(ms32, 4),
           "ms_fp32_top1": round(ms_top1, 4), "ms_fp64_map": round(ms64, 4),
           "fp32_map_evals_per_s": evals / (ms32 / 1e3),
           "fp32_top1_evals_per_s": evals / (ms_top1 / 1e3),
           "plain_fp64_evals_per_s": evals / (ms64 / 1e3),
           "speedup_fp32_top1_vs_plain_fp64": round(ms64 / ms_top1, 2),
           "ms_map_from_frame": forms,
           "fp32_vs_gpu_fp64_max_abs_drho": float(np.abs(g32 - g64).max())}
    if full_oracle:
        want = _oracle_map(ex, n_proc, f, ta)
        margin = O.top2_margin(want)
        u, v, r = O.argmax(want)
        out.update({"oracle": "whole map",
                    "fp32_max_abs_drho": float(np.abs(g32 - want).max()),
                    "fp64_max_abs_drho": float(np.abs(g64 - want).max()),
                    "oracle_argmax": [u, v], "oracle_top2_margin": margin,
                    "argmax_fp32_map": list(map(int, a32)), "argmax_fp64_map": list(map(int, a64)),
                    "argmax_fp32_top1": [int(b1["u"]), int(b1["v"])],
                    "argmax_match": bool(margin <= 1e-4 or (
                        tuple(a32) == tuple(a64) == (u, v) == (int(b1["u"]), int(b1["v"]))))})
    else:
        rng = np.random.default_rng(77)
        us, vs = rng.integers(0, nu, 4000), rng.integers(0, nv, 4000)
        extra = [(int(c[0]) + du, int(c[1]) + dv) for c in (a32, a64)
                 for du in range(-2, 3) for dv in range(-2, 3)]
        extra = [(a, b) for a, b in extra if 0 <= a < nu and 0 <= b < nv]
        us = np.concatenate([us, [a for a, _ in extra]])
        vs = np.concatenate([vs, [b for _, b in extra]])
        tables = O.sum_tables(f)
        want = O.rho_at(*tables, ta, us, vs)
        out.update({"oracle": f"{len(us)} offsets (4000 seeded + the neighbourhoods of the "
                              "GPU's best offsets)",
                    "fp32_max_abs_drho": float(np.abs(g32[vs, us] - want).max()),
                    "fp64_max_abs_drho": float(np.abs(g64[vs, us] - want).max()),
                    "argmax_fp32_map": list(map(int, a32)), "argmax_fp64_map": list(map(int, a64)),
                    "argmax_fp32_top1": [int(b1["u"]), int(b1["v"])],
                    "argmax_match": bool(tuple(a32) == tuple(a64) ==
                                         (int(b1["u"]), int(b1["v"])))})
    return out


def run_configs(S, torch, ctx, args):
    """The single-frame configurations (640x480 with a 32x32 template at
    sigma 8; 1920x1080 with a 64x64 template at sigma 4, 8, 16; 3840x2160
    textures with 128x128 and 256x256 templates at sigma 4, K_max 5000, and
    the 128x128 one uncapped) and the 16 x 64 batch (top-5), each with its
    FP32 throughput, the plain FP64 form's, and its error against the oracle."""
    from concurrent.futures import ProcessPoolExecutor
    from workloads import synth
    n_proc = max(1, min(16, len(os.sched_getaffinity(0))))
    res = {}
    with ProcessPoolExecutor(max_workers=n_proc) as ex:
        cases = [("scene_640x480_t32_s8", synth.scene_640x480(), 8, 5000, True)]
        cases += [(f"scene_1920x1080_t64_s{sg}", synth.scene_1920x1080(sg), sg, 5000, True)
                  for sg in (4, 8, 16)]
        cases += [(f"texture_3840x2160_t{sz}_s4" + ("" if km == 5000 else "_uncapped"),
                   synth.texture_3840x2160(sz, k_max=km), 4, km, args.full_parity)
                  for sz, km in ((128, 5000), (256, 5000), (128, 10 ** 9))]
        for name, wl, sg, km, full in cases:
            t0 = time.perf_counter()
            res[name] = _single_config(S, torch, ctx, ex, n_proc, wl, sg, km, full)
            log(f"[bench] {name}: {res[name]} ({time.perf_counter() - t0:.1f} s)")
    # the 16 x 64 batch: one tuned graph launch per step, against the plain form
    wl = synth.batch_16x64()
    B, N, M = len(wl.frames), wl.N, wl.M
    segs = [S.sncc_segment_template(t, sg, wl.k_max)[0] for t, sg in zip(wl.templates, wl.sigmas)]
    Kc = [len(a) for a in segs]
    tm = S.sncc_upload_templates(ctx, segs, [t.shape[1] for t in wl.templates],
                                 [t.shape[0] for t in wl.templates])
    f = torch.from_numpy(__import__("numpy").stack(wl.frames)).cuda()
    P = S.sncc_sat_pitch(M)
    s = torch.empty((B, N + 1, P), dtype=torch.int32, device="cuda")
    s2 = torch.empty_like(s)
    n = len(wl.pairs)
    topk = torch.zeros((n, wl.k, 3), dtype=torch.int32, device="cuda")
    batch = S.sncc_batch_create(ctx, tm, s, s2, B, M, N, wl.pairs, wl.k, topk, frames=f,
                                tune=args.tune, tune_cache=args.tune_cache)
    ms_step = _events_ms(torch, batch.run, 5)
    st = batch.stats()
    evals = st["coarse_evals"]
    out64 = torch.zeros_like(topk)
    ms64 = _events_ms(torch, lambda: S.sncc_topk(ctx, tm, s, s2, B, M, N, wl.pairs, wl.k,
                                                 S.SNCC_FP64, out64), 1)
    batch.run()
    torch.cuda.synchronize()
    g_top = [[(int(m["u"]), int(m["v"]), float(m["rho"])) for m in row]
             for row in S.decode_matches(topk)]
    cpu, parity = cpu_baseline(wl, Kc, budget_s=min(8.0, args.cpu_budget), gpu_topk=g_top)
    res["batch_16x64_top5"] = {
        "frames": B, "templates": len(wl.templates), "pairs": n, "K": [min(Kc), max(Kc)],
        "evals": evals, "ms_step": round(ms_step, 3), "ms_score": st["ms_score"],
        "evals_per_s": evals / (ms_step / 1e3), "frames_per_s": B / (ms_step / 1e3),
        "tile": f"{st['tile_u']}x{st['tile_v']}", "plain_fp64_ms": round(ms64, 3),
        "plain_fp64_evals_per_s": evals / (ms64 / 1e3),
        "speedup_vs_plain_fp64": round(ms64 / ms_step, 2),
        "cpu_oracle_evals_per_s": cpu["value"], "parity": parity}
    log(f"[bench] batch_16x64_top5: {res['batch_16x64_top5']}")
    batch.destroy()
    S.sncc_tmpl_destroy(tm)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="coarse-fine")
    ap.add_argument("--tune", type=int, default=1)
    ap.add_argument("--tune-cache", default=None,
                    help="JSON file of tuned tile configurations: read when it holds this "
                         "batch's key, else the tuner's choice is written to it")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--k", type=int, default=0, help="top-k per pair (default: the workload's)")
    ap.add_argument("--coarse-sigma", type=float, default=0,
                    help="override the coarse threshold of every template")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the per-configuration measurements (single frames, 16x64 batch)")
    ap.add_argument("--full-parity", action="store_true",
                    help="whole oracle maps for the 3840x2160 configurations too (minutes)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first copy a buffer of this size (a known-size kernel for "
                         "scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("this benchmark measures one GPU only: run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload == "threshold":
        run_threshold(args)
        return
    if args.workload == "prep":
        run_prep(args)
        return

    import numpy as np
    import torch
    import paper_2502_01286_amd as S

    if args.copy_calibration_mib:
        n = args.copy_calibration_mib << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda:0").fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] copied {args.copy_calibration_mib} MiB")
        del a, b
    log(f"[bench] generating workload {args.workload}")
    t0 = time.perf_counter()
    wl = make_workload(args.workload)
    if args.k:
        wl.k = args.k
    if args.coarse_sigma:
        wl.sigmas = [args.coarse_sigma] * len(wl.templates)
    B, N, M = len(wl.frames), wl.N, wl.M
    log(f"[bench] {B} frames {M}x{N}, {len(wl.templates)} templates, {len(wl.pairs)} pairs "
        f"({time.perf_counter() - t0:.1f} s)")

    # template preparation (host C++), reported separately
    t0 = time.perf_counter()
    coarse_l, fine_l = [], []
    for t, sg in zip(wl.templates, wl.sigmas):
        coarse_l.append(S.sncc_segment_template(t, sg, wl.k_max)[0])
        if wl.fine_sigma:
            fine_l.append(S.sncc_segment_template(t, wl.fine_sigma, wl.k_max)[0])
    prep_ms = (time.perf_counter() - t0) * 1e3
    Kc = [len(a) for a in coarse_l]
    log(f"[bench] prep {prep_ms:.1f} ms, K coarse {min(Kc)}..{max(Kc)}"
        + (f", K fine {min(map(len, fine_l))}..{max(map(len, fine_l))}" if fine_l else ""))

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ctx = S.sncc_ctx_create(0)
    Ws = [t.shape[1] for t in wl.templates]
    Hs = [t.shape[0] for t in wl.templates]
    coarse = S.sncc_upload_templates(ctx, coarse_l, Ws, Hs)
    fine = S.sncc_upload_templates(ctx, fine_l, Ws, Hs) if fine_l else None
    f = torch.from_numpy(np.stack(wl.frames)).to(dev)
    P = S.sncc_sat_pitch(M)
    s = torch.empty((B, N + 1, P), dtype=torch.int32, device=dev)
    s2 = torch.empty_like(s)
    n_pairs = len(wl.pairs)
    topk = torch.zeros((n_pairs, wl.k, 3), dtype=torch.int32, device=dev)
    best = torch.zeros((n_pairs, 4), dtype=torch.int32, device=dev) if fine else None
    cnt = torch.zeros(n_pairs, dtype=torch.int32, device=dev) if fine else None
    t0 = time.perf_counter()
    batch = S.sncc_batch_create(ctx, coarse, s, s2, B, M, N, wl.pairs, wl.k, topk, fine=fine,
                                radius=2, best_out=best, count_out=cnt, frames=f,
                                tune=args.tune, tune_cache=args.tune_cache)
    st = batch.stats()
    log(f"[bench] batch planned in {time.perf_counter() - t0:.2f} s: {st['work_items']} items, "
        f"tile {st['tile_u']}x{st['tile_v']}, {st['wg_threads']} threads, LDS {st['lds_bytes']} B, "
        f"{st['n_passes']} LDS passes over {len(wl.templates)} templates, computed/valid evals "
        f"{st['computed_evals'] / max(1, st['coarse_evals']):.3f}")

    for i in range(args.warmup):
        batch.run()
        torch.cuda.synchronize()
    log(f"[bench] warmup done")

    stages = {k: [] for k in ("ms_sat", "ms_score", "ms_select", "ms_refine", "ms_total")}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        batch.run()
        torch.cuda.synchronize()
        st = batch.stats()
        for k in stages:
            stages[k].append(st[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / args.steps
    avg = {k: (float(np.mean(v)) if v and min(v) >= 0 else None) for k, v in stages.items()}
    log(f"[bench] {args.steps} steps: {ms_per_step:.3f} ms/step, stages {avg}")
    evals = st["coarse_evals"]
    fine_offsets = int(cnt.sum().item()) if cnt is not None else 0
    value = evals / (ms_per_step / 1e3)

    roof = None
    if avg["ms_score"]:
        ops_tops = OPS_PER_EVAL * evals / (avg["ms_score"] / 1e3) / 1e12
        lds_tbs = 16 * evals / (avg["ms_score"] / 1e3) / 1e12
        roof = {"bound": "alu", "achieved": round(ops_tops, 3), "peak": round(VALU_PEAK_TOPS, 2),
                "unit": "TOP/s (VALU lane ops)", "frac": round(ops_tops / VALU_PEAK_TOPS, 4),
                "traffic": load_traffic(args.workload),
                "kernel": "tile_kernel (scoring stage: %d launch%s)"
                          % (st["n_launch_classes"], "es" if st["n_launch_classes"] > 1 else ""),
                "kernel_ms": round(avg["ms_score"], 4),
                "ops_per_eval": OPS_PER_EVAL, "evals_per_launch": evals,
                "lds": {"achieved_TBps": round(lds_tbs, 3), "peak_TBps": round(LDS_PEAK_TBS, 2),
                        "frac": round(lds_tbs / LDS_PEAK_TBS, 4), "bytes_per_eval": 16,
                        "peak_form": "ds_read_b128 (measured)",
                        "read2st64_TBps": round(LDS_READ2ST64_TBS, 2),
                        "frac_of_read2st64": round(lds_tbs / LDS_READ2ST64_TBS, 4)}}
        if avg.get("ms_refine") and cnt is not None:
            # FP64 re-score (steps 7f-i): unique neighbourhood offsets of each
            # pair x the fine approximation's segments, 5 method ops per eval
            # (as for the slow pass of the two-threshold search)
            Kf = [len(a) for a in fine_l]
            per_pair = cnt.cpu().numpy().astype(np.int64)
            fine_evals = int(sum(int(c) * Kf[t] for c, (_, t) in zip(per_pair, wl.pairs)))
            rtops = 5 * fine_evals / (avg["ms_refine"] / 1e3) / 1e12
            roof["refine"] = {"bound": "alu", "unit": "TOP/s (FP64 VALU lane ops)",
                              "achieved": round(rtops, 3), "peak": round(FP64_VALU_PEAK_TOPS, 2),
                              "frac": round(rtops / FP64_VALU_PEAK_TOPS, 4),
                              "ops_per_eval": 5, "evals": fine_evals,
                              "ms": round(avg["ms_refine"], 4)}
        if avg["ms_sat"]:
            px = B * M * N
            roof["sat"] = {"bound": "hbm", "achieved_GBps": round(9 * px / (avg["ms_sat"] / 1e3) / 1e9, 1),
                           "peak_GBps": 8000, "bytes_per_px": 9, "ms": round(avg["ms_sat"], 4)}

    plain = None
    if not args.no_plain:
        log("[bench] plain FP64 comparator (one launch per pair)")
        out64 = torch.zeros_like(topk)
        S.sncc_topk(ctx, coarse, s, s2, B, M, N, wl.pairs, wl.k, S.SNCC_FP64, out64)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 2
        e0.record()
        for _ in range(reps):
            S.sncc_topk(ctx, coarse, s, s2, B, M, N, wl.pairs, wl.k, S.SNCC_FP64, out64)
        e1.record()
        torch.cuda.synchronize()
        pms = e0.elapsed_time(e1) / reps
        plain = {"value": evals / (pms / 1e3), "unit": UNIT, "ms": round(pms, 3),
                 "speedup_batched_fp32": round((evals / (avg["ms_score"] / 1e3)) / (evals / (pms / 1e3)), 3)
                 if avg["ms_score"] else None,
                 "form": "one plain FP64 scoring launch per pair (+ per-pair top-k), no graph"}
        log(f"[bench] plain {pms:.2f} ms")

    cpu = parity = None
    if not args.no_cpu:
        log("[bench] CPU oracle baseline")
        g_top = S.decode_matches(topk)
        g_top = [[(int(m["u"]), int(m["v"]), float(m["rho"])) for m in row] for row in g_top]
        g_best = None
        if best is not None:
            g_best = [(int(m["u"]), int(m["v"]), float(m["rho"])) for m in S.decode_matches64(best)]
        cpu, parity = cpu_baseline(wl, Kc, budget_s=args.cpu_budget, gpu_topk=g_top,
                                   gpu_best=g_best)
        log(f"[bench] cpu {cpu}")
        log(f"[bench] parity on the oracle's sample {parity}")

    batch.destroy()
    S.sncc_tmpl_destroy(coarse)
    if fine:
        S.sncc_tmpl_destroy(fine)
    configs = None
    if not args.no_configs and args.workload == "coarse-fine":
        log("[bench] per-configuration measurements")
        configs = run_configs(S, torch, ctx, args)
    S.sncc_ctx_destroy(ctx)

    line = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "frames": B, "width": M, "height": N,
                   "templates": len(wl.templates), "pairs": n_pairs, "top_k": wl.k,
                   "coarse_sigma": sorted(set(wl.sigmas)), "fine_sigma": wl.fine_sigma,
                   "K_coarse": [min(Kc), max(Kc)], "coarse_evals": evals,
                   "fine_offsets_scored": fine_offsets,
                   "arith": "u32 box sums, i64 window energy, f32 compensated accumulation "
                            "and f32 rho (coarse), f64 refine"},
        "frames_per_s": B / (ms_per_step / 1e3),
        "stage_ms": avg, "prep_ms_host": prep_ms,
        "roofline": roof, "plain_fp64": plain, "cpu_baseline": cpu, "parity": parity,
        "configs": configs,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
