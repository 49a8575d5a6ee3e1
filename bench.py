#!/usr/bin/env python3
"""Throughput of the GLD time step on one MI355X.

Workload (default): N = 2e5 particles at density 0.5 (about 262 neighbours
within r_c = 5), memory m_max = 1000, dt = 0.01, WCA + exp-cos self and pair
memory (see paper_1808_00270_amd/workloads.py).  One "step" is the whole hot
path: neighbour build + F^C, history convolution, dissipative pair
contraction, colored noise (filter bank + Chebyshev mat-vec chain), update.

Prints ONE JSON line: whole-step particle-steps/s of the FP32-mixed path
(value), the FP64 path beside it, per-step latency p50/p99, per-kernel event
timings, the roofline of the dominant kernel and of the history convolution,
and the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_PEAK_TFLOPS = 157.3       # vector FP32
FP64_PEAK_TFLOPS = 78.6        # vector FP64
FP64_MATRIX_PEAK_TFLOPS = 78.6 # FP64 matrix cores (dense)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic(info, n, m_max, pairs, fp64, kind):
    """Algorithmic bytes (or flops) of one launch of a kernel class."""
    sT = 8 if fp64 else 4
    ib = info.get("list_index_bits", 16) / 8  # bytes per staged index in the lists
    # bytes per weight: 20-bit fixed point in the packed lists, which only the
    # cells with 12-bit indices hold (with some 16-bit cells, the full width)
    wb = info.get("list_weight_bits", 8 * sT) / 8 if ib == 1.5 else sT
    vec = 3 * n
    if kind == "history":
        # what the convolution of the definition streams per step: the ring,
        # the velocity, two outputs (the blocked form reads the ring once per
        # block instead)
        return dict(bytes=(m_max - 1) * vec * sT + vec * 8 + 2 * vec * sT)
    if kind == "dissipative":
        # staged index (12 or 16 bits) + weight per ordered pair, the pair
        # counts, the input vector once, the self-memory term added, the output
        return dict(bytes=pairs * (ib + wb) + 4 * n + vec * sT * 3)
    if kind == "noise_spmv":
        # a term that streams the pair lists: index (12 or 16 bits) + weight
        # per ordered pair, the pair counts, the input vector once, the
        # combination inputs z and the premixed v_k, the output (sorted T4
        # vectors: 4 components of sizeof(T)); the chain's first term has no
        # pair term and reads v_k only.  Arithmetic: 3 multiply-adds per
        # ordered pair (isotropic tensor) and the epilogue's 4 per component
        full = pairs * (ib + wb) + 4 * n + 4 * n * sT * (1 + 1 + 1 + 1)
        first = 4 * n * sT * 2
        return dict(full=full, first=first, flops=6.0 * pairs + 2.0 * 4 * vec)
    if kind == "noise_fir":
        P = 2 * info["window_half"] + 1
        # per step: a 1/block share of the block's outputs, block * rank
        # filters of P taps (the window kept by the noise plan) on 3N channels
        return dict(flops=2.0 * vec * info["rank"] * P)
    return {}


def run_gpu(args, fp64, window=1):
    import torch
    import paper_1808_00270_amd as pkg
    from paper_1808_00270_amd import workloads as wl

    w = wl.config(args.config)
    tag = ("fp64" if fp64 else "fp32-mixed") + (f", noise window {window}" if window > 1 else "")
    log(f"[bench] create {w.name} {tag}")
    t0 = time.perf_counter()
    s = pkg.System.from_workload(w, fp64=fp64, noise_window=window, verlet_skin=args.skin,
                                 rebuild_period=args.rebuild_period)
    t_create = time.perf_counter() - t0
    info = s.noise_info()
    log(f"[bench] created in {t_create:.1f}s, noise {info}")
    if args.no_graph:
        s.set_graph(False)
    # the lattice start melts over the first ~100 steps (list lengths and
    # the noise plan's choice settle); run it in untimed before the warmup
    s.step(args.equilibrate)
    s.sync()
    # warmup
    s.step(args.warmup)
    s.sync()
    # timed region: graph replay of K steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(args.steps)
    s.sync()
    torch.cuda.synchronize()
    dt_run = time.perf_counter() - t0
    ms_per_step = 1e3 * dt_run / args.steps
    log(f"[bench] {tag}: {ms_per_step:.3f} ms/step over {args.steps} steps")
    step_now = args.equilibrate + args.warmup + args.steps
    # whole spectrum-check cycles (the check runs every 100 steps): from the
    # next multiple of 100, `cycle_steps` steps timed the same way
    ms_cycle = None
    if args.cycle_steps > 0:
        s.step((-step_now) % 100)
        s.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(args.cycle_steps)
        s.sync()
        torch.cuda.synchronize()
        ms_cycle = 1e3 * (time.perf_counter() - t0) / args.cycle_steps
        log(f"[bench] {tag}: {ms_cycle:.3f} ms/step over {args.cycle_steps} steps from a check")
    # per-step latency, synchronous single steps
    lat = []
    for _ in range(args.latency_steps):
        t1 = time.perf_counter()
        s.step(1)
        s.sync()
        lat.append(1e3 * (time.perf_counter() - t1))
    # per-kernel durations with HIP events on the system's stream (same work),
    # and how many of those steps' chains used the tight noise plan
    tight0 = s.noise_info()["tight_steps"]
    s.set_timing(True)
    s.step(args.kernel_steps)
    kt = s.kernel_times()
    s.set_timing(False)
    after = s.noise_info()
    kt_tight = after["tight_steps"] - tight0
    # the index width of the lists those steps streamed (12 bits while every
    # cell's stencil holds at most 4096 particles)
    info["list_index_bits"] = max(info["list_index_bits"], after["list_index_bits"])
    info["theta_min"] = after["theta_min"]
    pairs, most = s.list_stats()
    st = s.read_state()
    s.close()
    del s
    torch.cuda.empty_cache()
    return dict(w=w, info=info, ms_per_step=ms_per_step, ms_cycle=ms_cycle, lat=lat, kt=kt, kt_tight=kt_tight,
                pairs=pairs, max_pairs=most, t_create=t_create, status=st["status"], window=window)


def measured_traffic(workload, kind, fp64):
    """Calibrated HBM bytes per launch of a kernel class from the committed
    rocprofv3 counter summary of this workload (profiles/*_traffic.json), or
    None when there is none or the kernel sources changed since it was taken."""
    import glob
    from paper_1808_00270_amd.profile_summary import source_hash
    cls = {"neighbor": "neighbor_build"}.get(kind, kind)
    tag = "fp64" if fp64 else "fp32"
    h = source_hash()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.json"))):
        with open(path) as f:
            d = json.load(f)
        if workload not in d.get("name", "") or not d["name"].endswith(tag):
            continue
        if d.get("source_sha256") != h:
            continue
        k = d.get("kernels", {}).get(cls)
        if k:
            return k["traffic_bytes"]
    return None


def pct(lat):
    if not lat:
        return None
    return {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))}


def roofline_entry(res, kind, fp64, kernel_steps):
    w, info = res["w"], res["info"]
    ms, cnt = res["kt"][kind]
    if cnt == 0:
        return None
    if kind == "history":
        # every step: a 1/HB share of the next block's matrix-core product (the
        # lags m > j + HB of its steps) and the step's own lags (m <= j + HB);
        # the ring is read once per block of HB steps
        hb = 16 if fp64 else 32
        per = ms / kernel_steps
        sT = 8 if fp64 else 4
        vec = 3 * w.n
        span = max(0, w.m_max - 1 - hb)
        flops = 2.0 * 2 * span * vec           # (K^s, g) rows x window x channels, per step (1/HB of HB rows)
        ring_bytes = span * vec * sT / hb      # the ring's share read by the product per step
        own = (hb + (hb - 1) / 2) * vec * sT   # the step's own lags, on average
        b = algorithmic(info, w.n, w.m_max, res["pairs"], fp64, kind)["bytes"]
        return dict(kernel=kind, method="blocked: a 1/HB share of the next block's matrix-core product every step "
                    "+ the step's own lags", block_steps=hb, ms_per_step=per,
                    matrix_flops_per_step=flops, matrix_tflops=flops / (per * 1e-3) / 1e12,
                    matrix_peak_tflops=FP64_MATRIX_PEAK_TFLOPS if fp64 else FP32_PEAK_TFLOPS,
                    hbm_bytes_per_step=ring_bytes + own + 8 * vec,
                    hbm_GBps=(ring_bytes + own + 8 * vec) / (per * 1e-3) / 1e9,
                    definition_bytes_per_step=b,
                    note="the per-step definition would stream definition_bytes_per_step; the blocked form "
                         "reads hbm_bytes_per_step")
    alg = algorithmic(info, w.n, w.m_max, res["pairs"], fp64, kind)
    if kind == "noise_fir":
        avg = ms / cnt
        fl = alg["flops"]
        ach = fl / (avg * 1e-3) / 1e12
        peak = FP64_MATRIX_PEAK_TFLOPS if fp64 else FP32_PEAK_TFLOPS
        return dict(kernel=kind, bound="mfma", achieved=ach, peak=peak, unit="TFLOP/s", frac=ach / peak,
                    traffic=None, avg_ms=avg, launches=cnt, flops_per_launch=fl)
    if kind == "noise_spmv":
        # the library times the chain's terms that stream the pair lists
        # between one event pair and counts them (the plan choice, skipped
        # terms and first term go to noise_setup).  With the per-step chain
        # and the isotropic tensor the first of them also computes P Y: its
        # extra vectors (Y and Dneg read, F^D' written: 10 n sizeof(T) per
        # step) are spread over the step's launches
        avg = ms / cnt
        b = alg["full"]
        if res.get("window", 1) == 1 and not w.parallel:
            b += 10 * w.n * (8 if fp64 else 4) * kernel_steps / cnt
    else:
        avg = ms / cnt
        b = alg["bytes"]
    ach = b / (avg * 1e-3) / 1e9
    out = dict(kernel=kind, bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
               traffic=measured_traffic(w.name, kind, fp64), avg_ms=avg, launches=cnt, bytes_per_launch=b,
               pairs=res["pairs"])
    if "flops" in alg:
        # the same launches against the vector FP32/FP64 peak (what the
        # mat-vec computes: 3 multiply-adds per ordered pair)
        tf = alg["flops"] / (avg * 1e-3) / 1e12
        peak = FP64_PEAK_TFLOPS if fp64 else FP32_PEAK_TFLOPS
        out["flop_view"] = dict(flops_per_launch=alg["flops"], achieved_tflops=tf, peak_tflops=peak,
                                frac=tf / peak)
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args):
    """The FP64 oracle on a bounded sample of the same workload: dissipative and
    conservative forces for a sample of particles, the colored noise for a
    subset of the frequencies of Algorithm 1; scaled to one full step.  Timed
    on all the host's cores and on one."""
    import oracle
    from paper_1808_00270_amd import workloads as wl

    w = wl.config(args.config)
    k_self, g, wt, r0, dr = w.tables()
    o = oracle.Oracle(n=w.n, box=w.box, dt=w.dt, mass=w.mass, kT=w.kT, k_self=k_self, k_pair=np.outer(wt, g),
                      r0=r0, dr=dr, r_cut=w.r_cut, wca_sigma=w.wca_sigma, wca_eps=w.wca_eps, seed=w.seed)
    R, V = w.initial_state()
    hist = np.zeros((w.m_max - 1, w.n, 3))   # zero pages; the oracle loops over every lag regardless
    rng = np.random.default_rng(0)

    def sample(rows_n, nw):
        rows = np.sort(rng.choice(w.n, size=rows_n, replace=False))
        t0 = time.perf_counter()
        o.forces_rows(R, V, hist, rows)
        t_rows = time.perf_counter() - t0
        t0 = time.perf_counter()
        o.noise(0, R, w0=0, w1=nw)
        t_noise = time.perf_counter() - t0
        return t_rows, t_noise, t_rows * (w.n / rows_n) + t_noise * (w.m_max / nw)

    cores = oracle.num_threads()
    t_rows, t_noise, t_step = sample(args.cpu_rows, args.cpu_freqs)
    oracle.set_threads(1)
    t1_rows, t1_noise, t1_step = sample(max(50, args.cpu_rows // 8), max(1, args.cpu_freqs // 8))
    oracle.set_threads(cores)
    return dict(value=w.n / t_step, unit="particle-steps/s", cores=cores, kind="oracle",
                sample=(f"{w.name}: F^C+F^D' of {args.cpu_rows} random particles ({t_rows:.1f}s) and the "
                        f"Algorithm-1 noise for {args.cpu_freqs} of {w.m_max} frequencies incl. pair search "
                        f"({t_noise:.1f}s), scaled to one full step = {t_step:.0f}s"),
                seconds=t_rows + t_noise + t1_rows + t1_noise, cpu_model=cpu_model(), build="gcc -O3 -fopenmp",
                single_core=dict(value=w.n / t1_step, unit="particle-steps/s", cores=1,
                                 sample=(f"F^C+F^D' of {max(50, args.cpu_rows // 8)} particles ({t1_rows:.1f}s), "
                                         f"noise for {max(1, args.cpu_freqs // 8)} frequencies ({t1_noise:.1f}s), "
                                         f"scaled to one full step = {t1_step:.0f}s")))


def run_batch(args):
    """The batched workload: 256 independent systems (N log-uniform in
    [100, 2e4], density in [0.005, 0.5], m_max in {200, 500, 1000}, kernels
    scaled by factors in [0.5, 2]) in one batch, FP32-mixed, one graph replay
    per step for all of them, mat-vec schedule from the autotuner."""
    import torch
    from paper_1808_00270_amd import batch as bm
    from paper_1808_00270_amd import workloads as wl

    t0 = time.perf_counter()
    b = bm.Batch(args.batch_systems, args.batch_gib << 30, fp64=False)
    attempts = [0] * args.batch_systems
    pending = list(range(args.batch_systems))
    slot_of = {}
    redrawn = 0
    for _ in range(12):
        if not pending:
            break
        ws = [wl.batch_system(i, attempts[i]) for i in pending]
        systems = []
        for w in ws:
            p, keep = bm.workload_params(w)
            R, V = w.initial_state()
            systems.append((p, keep, R, V))
        slots, stat = b.add(systems, strict=False)
        nxt = []
        for i, w, s, st in zip(pending, ws, slots, stat):
            if s >= 0:
                slot_of[i] = (s, w)
            else:
                if st == -5:
                    raise RuntimeError("batched workload does not fit the workspace")
                attempts[i] = w.attempt + 1   # not positive definite / outside the interval: draw again
                redrawn += 1
                nxt.append(i)
        pending = nxt
    t_setup = time.perf_counter() - t0
    n_tot = sum(w.n for s, w in slot_of.values())
    log(f"[bench] batch: {len(slot_of)} systems, {n_tot} particles, set up in {t_setup:.1f}s ({redrawn} redrawn)")
    thr, cand_ms = b.autotune(3)
    log(f"[bench] batch autotune: thresholds {thr}, ms per pass {[round(x, 3) for x in cand_ms]}")
    b.step(args.warmup)
    b.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(args.steps)
    b.sync()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.steps
    log(f"[bench] batch: {ms:.3f} ms/step")
    b.set_timing(True)
    b.step(args.batch_kernel_steps)
    kt = b.kernel_times()
    b.set_timing(False)
    nsys, npart, pairs = b.stats()
    bad = sum(1 for s, w in slot_of.values() if b.read_state(s)["flags"] != 0)
    # the chain's list streams: per system K - 1 Clenshaw mat-vecs plus the
    # dissipative one, each over its pairs (16-bit index + 32-bit weight)
    term_pairs, lanes_hist = 0, {}
    for s, w in slot_of.values():
        pr, ln = b.system_stats(s)
        K = b.noise_info(s)["cheb_terms"]
        term_pairs += pr * K
        lanes_hist[ln] = lanes_hist.get(ln, 0) + 1
    ring_bytes = sum(4 * 3 * w.n * (w.m_max - 1) for s, w in slot_of.values())
    per = {k: v / args.batch_kernel_steps for k, (v, c) in kt.items()}
    hist_ms = per["history"]
    b.close()
    del b
    torch.cuda.empty_cache()
    return {
        "workload": "batch256_n100-2e4_rho0.005-0.5_m200-1000",
        "systems": nsys, "particles": npart, "pairs": pairs, "redrawn": redrawn, "flagged_systems": bad,
        "value": npart * 1e3 / ms, "unit": "particle-steps/s", "ms_per_step": ms,
        "schedule_lane_thresholds": thr, "autotune_ms_per_candidate": cand_ms,
        "kernels_ms_per_step": per,
        "lanes_per_particle_systems": {str(k): v for k, v in sorted(lanes_hist.items())},
        "roofline_spmv": {"kernel": "noise_spmv (dissipative + Clenshaw mat-vecs of every system)", "bound": "hbm",
                          "pair_terms_per_step": term_pairs, "bytes_per_step": 6 * term_pairs,
                          "achieved": 6 * term_pairs / (per["noise_spmv"] * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": 6 * term_pairs / (per["noise_spmv"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                          "note": "list bytes only (index and weight per pair term); the vectors come from L2"},
        "roofline_history": {"kernel": "history (streamed every step)", "bound": "hbm",
                             "bytes_per_step": ring_bytes + npart * 3 * (8 + 4 * 3),
                             "achieved": (ring_bytes + npart * 3 * (8 + 4 * 3)) / (hist_ms * 1e-3) / 1e9,
                             "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": (ring_bytes + npart * 3 * (8 + 4 * 3)) / (hist_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "setup_s": t_setup,
    }


def run_general(args):
    """The general memory model (rank-two pair table, Delta K^s, noise by
    Algorithm 1 per frequency on the GPU), FP64."""
    import torch
    from paper_1808_00270_amd import general
    from paper_1808_00270_amd import workloads as wl

    n, rho, M = args.general_n, args.general_rho, args.general_m
    w = wl.Workload(name=f"general_n{n}_rho{rho}_m{M}", n=n, rho=rho, m_max=M, steps=0, seed=3100)
    ks, kp, dks, r0, dr = wl.general_tables(M, 101, w.r_cut, w.dt)
    R, V = w.initial_state()
    log(f"[bench] general: create {w.name}")
    t0 = time.perf_counter()
    s = general.GeneralSystem(n=n, box=w.box, dt=w.dt, mass=w.mass, kT=w.kT, k_self=ks, k_pair=kp, dk_self=dks,
                              r0=r0, dr=dr, r_cut=w.r_cut, wca_sigma=w.wca_sigma, wca_eps=w.wca_eps, seed=w.seed,
                              r=R, v=V)
    t_create = time.perf_counter() - t0
    s.step(args.general_warmup)
    s.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(args.general_steps)
    s.sync()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.general_steps
    log(f"[bench] general: {ms:.3f} ms/step over {args.general_steps} steps")
    s.set_timing(True)
    s.step(args.general_kernel_steps)
    kt = s.kernel_times()
    s.set_timing(False)
    info = s.info()
    s.close()
    del s
    torch.cuda.empty_cache()
    per = {k: v / args.general_kernel_steps for k, (v, c) in kt.items()}
    cpu = None
    if not args.no_cpu:
        # the oracle on a sample of the same workload: F^C + F^D' of 500
        # particles and Algorithm 1 for 4 of the frequencies, scaled to a step
        import oracle
        o = oracle.Oracle(n=n, box=w.box, dt=w.dt, mass=w.mass, kT=w.kT, k_self=ks, k_pair=kp, dk_self=dks, r0=r0,
                          dr=dr, r_cut=w.r_cut, wca_sigma=w.wca_sigma, wca_eps=w.wca_eps, seed=w.seed,
                          lanczos_tol=1e-12)
        rows = np.sort(np.random.default_rng(0).choice(n, size=500, replace=False))
        hist = np.zeros((M - 1, n, 3))
        t0 = time.perf_counter()
        o.forces_rows(R, V, hist, rows)
        t_rows = time.perf_counter() - t0
        t0 = time.perf_counter()
        o.noise(0, R, w0=0, w1=4)
        t_noise = time.perf_counter() - t0
        t_step = t_rows * n / 500 + t_noise * M / 4
        cpu = {"value": n / t_step, "unit": "particle-steps/s", "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"F^C+F^D' of 500 particles ({t_rows:.1f}s) and Algorithm 1 for 4 of {M} frequencies "
                         f"({t_noise:.1f}s), scaled to one step = {t_step:.0f}s"}
        log(f"[bench] general: oracle sample {t_rows + t_noise:.1f}s, {t_step:.0f}s per step")
    lz = kt["lanczos"]
    lz_ms = lz[0] / max(lz[1], 1)
    # per frequency and Lanczos iteration the mat-vec streams the pair list
    # (j and the grid coordinate: 12 bytes a pair) and touches the Krylov vectors:
    # reads v and writes K v (mat-vec), reads K v, v_k, v_{k-1} and writes
    # v_{k+1} (recurrence and scaling, 2 passes), then reads the basis once
    # for x = |b| V y: (6 + 1) * 3n doubles; iterations counted at the last
    # step's largest dimension (an upper bound)
    k = info["last_iters"]
    lz_bytes = M * (k * (12 * info["pairs"] + 7 * 3 * n * 8) + 2 * 3 * n * 8)
    return {
        "workload": w.name, "n": n, "rho": rho, "m_max": M, "n_r": 101, "dtype": "f64",
        "value": n * 1e3 / ms, "unit": "particle-steps/s", "ms_per_step": ms, "create_s": t_create,
        "lanczos_max_dim_last_step": k, "pairs": info["pairs"], "max_per_particle": info["max_per_particle"],
        "cpu_baseline": cpu,
        "kernels_ms_per_step": per,
        "roofline_lanczos": {"kernel": "lanczos (one work-group per frequency)", "bound": "hbm",
                             "bytes_per_launch_upper": lz_bytes, "avg_ms": lz_ms,
                             "achieved": lz_bytes / (lz_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": lz_bytes / (lz_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                             "note": "pair list and Krylov vectors mostly served from L2/MALL; the byte count "
                                     "takes every iteration at the largest dimension"},
    }


def run_serve(args):
    """Continuous-batching server on the first requests of the serving
    workload (Poisson arrivals, uneven N, m_max and step counts scaled by
    --serve-steps-scale)."""
    import torch
    from paper_1808_00270_amd import batch
    from paper_1808_00270_amd import workloads as wl

    reqs = wl.serve_requests(args.serve_requests, steps_scale=args.serve_steps_scale)
    sv = batch.Server(args.serve_slots, args.serve_gib << 30, chunk_steps=args.serve_chunk)
    keep, ids = [], []
    for t, steps, w in reqs:
        p, k = batch.workload_params(w, fp64=False)
        R, V = w.initial_state()
        rid, foot = sv.submit(p, R, V, steps, t)
        ids.append((rid, w, steps))
        keep.append(k)
    log(f"[bench] serve: {len(reqs)} requests submitted")
    torch.cuda.synchronize()
    sv.run()
    makespan, bsteps = sv.stats()
    lat, queue, service, work, failed = [], [], [], 0, 0
    for rid, w, steps in ids:
        rec, _ = sv.request(rid, state=False)
        if rec["status"] != 0:
            failed += 1
            continue
        lat.append(1e3 * (rec["done_s"] - rec["arrival_s"]))
        queue.append(1e3 * (rec["admitted_s"] - rec["arrival_s"]))
        service.append(1e3 * (rec["done_s"] - rec["admitted_s"]))
        work += w.n * steps
    sv.close()
    del sv
    torch.cuda.empty_cache()
    log(f"[bench] serve: makespan {makespan:.2f}s, {bsteps} batch steps, {failed} refused")
    return {
        "workload": f"serve_poisson20_first{args.serve_requests}_steps_x{args.serve_steps_scale}",
        "requests": len(reqs), "served": len(lat), "refused": failed, "slots": args.serve_slots,
        "chunk_steps": args.serve_chunk, "makespan_s": makespan, "batch_steps": bsteps,
        "value": work / makespan, "unit": "particle-steps/s",
        "latency_ms": pct(lat), "queueing_ms": pct(queue), "service_ms": pct(service),
        "note": "arrivals at 20/s; each request's steps log-uniform in [1e3, 1e5] times the scale",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", type=int, default=3)
    ap.add_argument("--latency-steps", type=int, default=1000)
    ap.add_argument("--kernel-steps", type=int, default=100,
                    help="steps timed kernel by kernel (100: one spectrum check included)")
    ap.add_argument("--cycle-steps", type=int, default=200,
                    help="steps timed from a multiple of the check interval (whole check cycles); 0: skip")
    ap.add_argument("--cpu-rows", type=int, default=2000)
    ap.add_argument("--cpu-freqs", type=int, default=16)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--batch-systems", type=int, default=256, help="systems of the batched leg (0: skip)")
    ap.add_argument("--batch-gib", type=int, default=48, help="workspace of the batched leg, GiB")
    ap.add_argument("--batch-kernel-steps", type=int, default=10)
    ap.add_argument("--general-n", type=int, default=10000, help="particles of the general-model leg (0: skip)")
    ap.add_argument("--general-rho", type=float, default=0.05)
    ap.add_argument("--general-m", type=int, default=500)
    ap.add_argument("--general-steps", type=int, default=10)
    ap.add_argument("--general-warmup", type=int, default=2)
    ap.add_argument("--general-kernel-steps", type=int, default=3)
    ap.add_argument("--serve-requests", type=int, default=64, help="requests of the serving leg (0: skip)")
    ap.add_argument("--serve-steps-scale", type=float, default=0.01)
    ap.add_argument("--serve-slots", type=int, default=32)
    ap.add_argument("--serve-gib", type=int, default=32)
    ap.add_argument("--serve-chunk", type=int, default=50)
    ap.add_argument("--skin", type=float, default=0.6, help="Verlet skin of the single-system runs")
    ap.add_argument("--equilibrate", type=int, default=200,
                    help="untimed steps from the lattice start before the warmup (single-system runs)")
    ap.add_argument("--rebuild-period", type=int, default=20,
                    help="candidate-list rebuild cadence in steps (the displacement test stays as the safety "
                         "net; 0: the displacement test alone)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="launch every step eagerly (counter runs)")
    ap.add_argument("--window", type=int, default=8,
                    help="also time the FP32-mixed step with this noise window (the random forces of W steps "
                         "at the positions of the window's first step; 0 or 1: skip)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the runs, negate this many MiB of float32 once: a kernel of known HBM "
                         "traffic that calibrates the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this library runs one system on one GPU; multi-GPU runs are not supported "
              "(each GPU would take its own systems with no communication).", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)

    r32 = run_gpu(args, fp64=False)
    r64 = None if args.no_fp64 else run_gpu(args, fp64=True)
    rw = run_gpu(args, fp64=False, window=args.window) if args.window > 1 else None
    if args.calib_copy_mib > 0:
        nf = args.calib_copy_mib * (1 << 20) // 4
        a = torch.ones(nf, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.neg(a, out=b)
        torch.cuda.synchronize()
        log(f"[bench] calibration: negated {nf * 4} bytes (read {nf * 4}, write {nf * 4})")
        del a, b
    w = r32["w"]
    value = w.n * 1e3 / r32["ms_per_step"]
    per_step = {k: ms / args.kernel_steps for k, (ms, c) in r32["kt"].items()}
    dom = max((k for k in per_step if k != "check"), key=lambda k: per_step[k])
    roof = roofline_entry(r32, dom, False, args.kernel_steps)
    roof_hist = roofline_entry(r32, "history", False, args.kernel_steps)
    out = {
        "metric": "particle-steps/s, N=2e5, m_max=1000 (FP32-mixed vs FP64 plain); p50/p99 latency",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "rho": w.rho, "m_max": w.m_max, "r_cut": w.r_cut, "dt": w.dt,
                   "precision": "fp32-mixed (f32 history/noise, f64 positions and update)",
                   "verlet_skin": args.skin, "rebuild_period": args.rebuild_period},
        "latency_ms": pct(r32["lat"]),
        "noise": {k: r32["info"][k] for k in ("cheb_terms", "cheb_terms_tight", "lam_hi", "lam_hi_tight", "rank",
                                              "block", "window_half", "err_estimate", "list_index_bits",
                                              "list_weight_bits")}
                 | {"tight_fraction_kernel_steps": r32["kt_tight"] / args.kernel_steps},
        "kernels_ms_per_step": per_step,
        "roofline": {k: roof[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")}
                    | {"kernel": dom, "pairs": r32["pairs"], "avg_ms": roof["avg_ms"]}
                    | ({"flop_view": roof["flop_view"]} if "flop_view" in roof else {}),
        "roofline_history": roof_hist,
        "ms_per_step_whole_check_cycles": r32["ms_cycle"],
        "check_interval": 100,
        "pairs": {"directed": r32["pairs"], "per_particle": r32["pairs"] / w.n, "max_per_particle": r32["max_pairs"]},
    }
    if r64 is not None:
        out["fp64_plain"] = {
            "value": w.n * 1e3 / r64["ms_per_step"], "ms_per_step": r64["ms_per_step"],
            "ms_per_step_whole_check_cycles": r64["ms_cycle"],
            "latency_ms": pct(r64["lat"]),
            "noise": {k: r64["info"][k] for k in ("cheb_terms", "cheb_terms_tight", "rank", "block", "window_half",
                                                  "err_estimate", "list_index_bits", "list_weight_bits")}
                     | {"tight_fraction_kernel_steps": r64["kt_tight"] / args.kernel_steps},
            "kernels_ms_per_step": {k: ms / args.kernel_steps for k, (ms, c) in r64["kt"].items()},
            "roofline_history": roofline_entry(r64, "history", True, args.kernel_steps),
        }
        out["fp32_over_fp64"] = r64["ms_per_step"] / r32["ms_per_step"]
    if rw is not None:
        # a variant, not the headline: the exact method computes every step's
        # random force at that step's positions
        out["fp32_noise_window"] = {
            "window": args.window, "value": w.n * 1e3 / rw["ms_per_step"], "ms_per_step": rw["ms_per_step"],
            "speedup": r32["ms_per_step"] / rw["ms_per_step"],
            "noise": {k: rw["info"][k] for k in ("cheb_terms", "rank", "block", "noise_window")},
            "kernels_ms_per_step": {k: ms / args.kernel_steps for k, (ms, c) in rw["kt"].items()},
            "note": "random forces of W consecutive steps computed together at the positions of the window's "
                    "first step (the variant proposed for time-scale separation); not the per-step method",
        }
    if args.batch_systems > 0:
        rb = run_batch(args)
        rb["fp32_batched_over_fp64_single"] = rb["value"] / out["fp64_plain"]["value"] if r64 is not None else None
        out["batched"] = rb
    if args.general_n > 0:
        out["general"] = run_general(args)
    if args.serve_requests > 0:
        out["serving"] = run_serve(args)
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle sample)")
        out["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
