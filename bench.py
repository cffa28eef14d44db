#!/usr/bin/env python3
"""Benchmark of the KPM-DOS hot path on one MI355X.

Workload: the topological-insulator Hamiltonian on a periodic 64x64x64
lattice (N = 1,048,576 rows, 13 stored entries per row), disorder gamma = 1,
R = 32 random-phase start vectors, M = 2000 Chebyshev moments, complex128
storage, FP64 scalar products, Jackson-kernel DOS on 4096 energies.

One step = kpm_moments (1000 fused aug_spmmv sweeps, the deterministic
scalar-product reductions, the eta -> mu identity and the moment check) plus
kpm_dos, on a Hamiltonian and start block already resident in HBM.  The
metric is the paper's minimum traffic of the blocked sweep,
V = Nnz (S_d + S_i) + 3 R S_d N bytes per sweep, divided by the step time.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "aug_spmmv HBM GB/s (% peak) & Gflop/s; time-to-DOS at fixed L1 err, plain vs opt"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
WORKLOADS = {
    # name: (L, gamma, R, M, dtype, K)
    "ti64_r32_m2000_c128": ((64, 64, 64), 1.0, 32, 2000, "c128", 4096),
    "ti128x128x64_r32_m2000_c64": ((128, 128, 64), 2.0, 32, 2000, "c64", 4096),
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_traffic.json")
PROFILE_PERIOD = 8   # headline: one sweep launch in 8 is bracketed by HIP events
CSRC = os.path.join(ROOT, "paper_1410_5242_amd", "csrc")
# sources that define each sweep kernel (hashed to tie counters to the code they were taken on)
KERNEL_SOURCES = {
    "lattice_kernel": ["kpm_lattice.hip", "kpm_sweep.h"],
    "aug_spmmv_kernel": ["kpm_sweep.h", "kpm_sweep_c128_large.hip", "kpm_sweep_c64_large.hip"],
    "gather_sweep_kernel": ["kpm_gather.h", "kpm_batched.h", "kpm_gather_c128.hip", "kpm_gather_c64.hip"],
    "window_sweep_kernel": ["kpm_gather.h", "kpm_batched.h", "kpm_gather_c128.hip", "kpm_gather_c64.hip"],
}


def kernel_source_sha(kernel: str) -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def sweep_bytes(N, nnz, R, Sd, Si=4):
    """Minimum bytes per blocked sweep: Nnz (S_d + S_i) + 3 R S_d N."""
    return nnz * (Sd + Si) + 3 * R * Sd * N


def sweep_flops(N, R, nnzr=13, Fa=2, Fm=6):
    """Flops per sweep: R N [Nnzr (Fa + Fm) + ceil(7 Fa / 2) + ceil(9 Fm / 2)]."""
    return R * N * (nnzr * (Fa + Fm) + math.ceil(7 * Fa / 2) + math.ceil(9 * Fm / 2))


def traffic_record(kernel: str, workload: str):
    """Calibrated HBM bytes per launch from the committed rocprofv3 counters, or None when the
    counters were taken on another kernel source or workload."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    rec = json.load(open(TRAFFIC_FILE)).get(f"{kernel}:{workload}")
    if not rec or rec.get("source_sha256") != kernel_source_sha(kernel):
        return None
    return rec.get("hbm_bytes_per_launch")


def _oracle_sweeps_rate(Ho, a, b, v0, target_s, max_sweeps=512):
    """Seconds per sweep of the oracle's blocked recurrence, from as many sweeps as fit in about
    target_s (at least one, at most max_sweeps); returns (sweeps, seconds)."""
    import oracle as O
    t0 = time.perf_counter()
    O.kpm_eta(Ho, a, b, v0, 2)                 # one sweep (with the first touch of its buffers)
    t1 = time.perf_counter() - t0
    sweeps = int(max(1, min(max_sweeps, target_s / max(t1, 1e-3))))
    t0 = time.perf_counter()
    O.kpm_eta(Ho, a, b, v0, 2 * sweeps)
    return sweeps, time.perf_counter() - t0


def host_cores() -> dict:
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"cpu_count": os.cpu_count(), "affinity": aff, "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(L, gamma, R, dtype, target_s=15.0):
    """Time the plain CPU oracle on a bounded number of sweeps of the same workload, on all the
    threads the process may use (OMP_NUM_THREADS, else every core it may run on), then on one."""
    import oracle as O
    from paper_1410_5242_amd import inputs
    pot = inputs.potential(L, gamma, 0)
    Ho = O.ti_hamiltonian(L, pot)
    a, b = O.scaling(*O.gershgorin(Ho))
    v0 = inputs.phase_block(Ho.n, R, 0)
    Sd = 16  # the oracle always runs in complex128
    bps = sweep_bytes(Ho.n, 13 * Ho.n, R, Sd)
    cores = host_cores()
    threads = int(cores["OMP_NUM_THREADS"] or cores["affinity"])
    O.set_lib_threads(threads)
    threads = O.lib_threads()
    sweeps, dt = _oracle_sweeps_rate(Ho, a, b, v0, target_s)
    O.set_lib_threads(1)
    sweeps1, dt1 = _oracle_sweeps_rate(Ho, a, b, v0, target_s / 3)
    O.set_lib_threads(threads)
    return {"value": round(bps * sweeps / dt / 1e9, 3), "unit": "GB/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{sweeps} sweeps (M={2 * sweeps}) of the same lattice, R and seed, complex128, "
                      f"{dt:.2f} s on {threads} threads; Gflop/s {sweep_flops(Ho.n, R) * sweeps / dt / 1e9:.2f}",
            "host": cores,
            "single_thread": {"value": round(bps * sweeps1 / dt1 / 1e9, 3), "unit": "GB/s", "cores": 1,
                              "sample": f"{sweeps1} sweeps, {dt1:.2f} s"}}


def cpu_oracle_subsets(target_s=8.0):
    """The oracle on the small configuration in full (8^3, R = 1, M = 128) and on bounded subsets of the
    other workloads, extrapolated linearly (stated per entry): the 128 x 128 x 64 precision lattice
    (complex128, per sweep), the batched family (R = 8, M = 512, per instance) and the learned family's
    truth runs (R = 16, M = 4096, per instance)."""
    import numpy as np
    import oracle as O
    from paper_1410_5242_amd import inputs, learned
    out = {"threads": O.lib_threads()}
    L1, M1 = (8, 8, 8), 128
    t0 = time.perf_counter()
    H1 = O.ti_hamiltonian(L1, inputs.potential(L1, 1.0, 0))
    a1, b1 = O.scaling(*O.gershgorin(H1))
    v1 = inputs.phase_block(H1.n, 1, 0)
    build1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.kpm_moments(H1, a1, b1, v1, M1)
    run1 = time.perf_counter() - t0
    out["small_8x8x8_r1_m128"] = {"sample": "the full run", "seconds": round(run1, 4), "build_s": round(build1, 3),
                                  "GBps": round(sweep_bytes(H1.n, 13 * H1.n, 1, 16) * (M1 // 2) / run1 / 1e9, 2)}
    del H1, v1
    L, R = (128, 128, 64), 32
    pot = inputs.potential(L, 2.0, 0)
    t0 = time.perf_counter()
    Ho = O.ti_hamiltonian(L, pot)
    a, b = O.scaling(*O.gershgorin(Ho))
    build = time.perf_counter() - t0
    v0 = inputs.phase_block(Ho.n, R, 0)
    sweeps, dt = _oracle_sweeps_rate(Ho, a, b, v0, 2 * target_s, max_sweeps=20)
    bps = sweep_bytes(Ho.n, 13 * Ho.n, R, 16)
    out["precision_128x128x64_r32_m2000"] = {
        "sample": f"{sweeps} sweeps", "seconds_per_sweep": round(dt / sweeps, 4), "GBps": round(bps * sweeps / dt / 1e9, 2),
        "build_s": round(build, 2), "full_run_s_extrapolated": round(dt / sweeps * 1000, 1)}
    del Ho, v0
    for name, fam, Rf, M, n_total in (
            ("batched_512_r8_m512", inputs.instance_family(512, (12, 16, 20, 24), 4.0, 0), 8, 512, 512),
            ("learned_truth_r16_m4096", learned.family(22000, learned.TRAIN_SEED), 16, learned.M_TRUTH, 22000)):
        t_inst, done, t_start = [], 0, time.perf_counter()
        for f in fam:
            Hf = O.ti_hamiltonian(f["L"], inputs.potential(f["L"], f["gamma"], f["pot_seed"]))
            af, bf = O.scaling(*O.gershgorin(Hf))
            vf = inputs.phase_block(Hf.n, Rf, f["vec_seed"])
            t0 = time.perf_counter()
            O.kpm_eta(Hf, af, bf, vf, M)
            t_inst.append(time.perf_counter() - t0)
            done += 1
            if time.perf_counter() - t_start > target_s:
                break
        mean_n = float(np.mean([4 * f["L"][0] ** 3 for f in fam]))
        done_n = float(np.mean([4 * f["L"][0] ** 3 for f in fam[:done]]))
        per = float(np.mean(t_inst)) * mean_n / done_n
        out[name] = {"sample": f"first {done} of {n_total} instances at full M, R", "seconds_per_instance": round(per, 3),
                     "all_instances_s_extrapolated": round(per * n_total, 1),
                     "note": "per-instance time scaled by the family's mean N over the sample's mean N"}
    return out


def leg_precision(log_fn=None):
    """128 x 128 x 64 lattice, gamma = 2, R = 32, M = 2000: complex64 storage with FP64 products
    against complex128 on the same seed (moments error, DOS L1 error, speed)."""
    import numpy as np
    import torch
    from paper_1410_5242_amd import autotune, inputs, kpm
    L, gamma, R, M, K = (128, 128, 64), 2.0, 32, 2000, 4096
    pot = inputs.potential(L, gamma, 0)
    res = {"workload": f"TI {L[0]}x{L[1]}x{L[2]} periodic, gamma={gamma}, R={R}, M={M}, same potential and start "
                       f"vectors (complex64 block = rounded complex128 block), Jackson DOS on {K} energies"}
    mus, rhos, times = {}, {}, {}
    a = b = None
    for dt in ("c128", "c64"):
        H = kpm.build_hamiltonian(L, pot, dtype=dt)
        kpm.reset_sweep_tuning()
        tuned = autotune.apply_sweep(autotune.TuningCache(), H, R, L)
        a, b = H.a, H.b
        V0 = kpm.random_phase_block(H.N, R, 0, dt)
        E = torch.from_numpy(H.b + H.a * (-1.0 + (2.0 * np.arange(K) + 1.0) / K)).cuda()
        mu = kpm.moments(H, V0, M)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        kpm.moments(H, V0, M, mu=mu)
        rho = kpm.dos(mu, H.a, H.b, E)
        ev[1].record()
        torch.cuda.synchronize()
        times[dt] = ev[0].elapsed_time(ev[1]) / 1e3
        mus[dt], rhos[dt] = mu.cpu().numpy(), rho.cpu().numpy()
        Sd = 16 if dt == "c128" else 8
        bps = sweep_bytes(H.N, 13 * H.N, R, Sd)
        res[dt] = {"seconds": round(times[dt], 4), "GBps": round(bps * (M // 2) / times[dt] / 1e9, 1),
                   "sweep_kernel": kpm.sweep_kernel(H, R), "autotuned": tuned}
        kpm.reset_sweep_tuning()
        H.close()
        del V0
    dE = 2.0 * a / K
    # against the FP64 oracle: its first 400 moments (200 sweeps) of this lattice, seed and start
    # block, stored by tests/golden/make_oracle_moments.py
    gold = os.path.join(ROOT, "tests", "golden", "ti128x128x64_g2_r32_m400_mu.npy")
    if os.path.exists(gold):
        ref = np.load(gold, allow_pickle=False)
        Mp = ref.shape[1]
        res["vs_oracle_prefix"] = {"moments": Mp, "sweeps": Mp // 2,
                                   "c128_max_abs_mu_error": float(np.abs(mus["c128"][:, :Mp] - ref).max()),
                                   "c64_max_abs_mu_error": float(np.abs(mus["c64"][:, :Mp] - ref).max()),
                                   "c64_mean_abs_mu_error": float(np.abs(mus["c64"][:, :Mp] - ref).mean())}
    d = np.abs(mus["c64"] - mus["c128"])
    res["max_abs_mu_error"] = float(d.max())
    res["mean_abs_mu_error"] = float(d.mean())
    res["dos_l1_error"] = float(np.abs(rhos["c64"] - rhos["c128"]).sum() * dE)
    res["stated_bound"] = {"max_abs_mu_error": 1e-5, "dos_l1_error": 1e-5}
    res["within_bound"] = bool(res["max_abs_mu_error"] <= 1e-5 and res["dos_l1_error"] <= 1e-5)
    res["speedup_c64"] = round(times["c128"] / times["c64"], 3)
    return res


def leg_stream(nbytes: int = 4 << 30, reps: int = 5):
    """Attainable HBM bandwidth b, the bound the paper measures for each machine (Table
    "tab:architectures", eq. "eq:roofline_mem"): the library's STREAM read, copy and triad kernels
    on arrays 16 times the last-level cache, best launch over workgroups per CU and load / store
    hint.  b is the highest of the three: what the memory delivers to a kernel of ours."""
    import torch
    from paper_1410_5242_amd import kpm
    n = nbytes // 8
    a = torch.full((n,), 1.0, dtype=torch.float64, device="cuda")
    b = torch.full((n,), 2.0, dtype=torch.float64, device="cuda")
    c = torch.empty_like(a)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    part = torch.zeros(cus * 8, dtype=torch.float64, device="cuda")
    out = {"workload": f"{nbytes >> 30} GiB FP64 arrays, 256-thread workgroups, best of {reps} launches per shape; "
                       "read moves 1x, copy 2x, triad 3x the array bytes", "points": []}
    best = {}
    for kind, traffic in (("read", nbytes), ("copy", 2 * nbytes), ("triad", 3 * nbytes)):
        for wg in (1, 2, 4, 8):
            for nt in (False, True):
                if kind == "read":
                    part.zero_()
                    args = (kind, part, a, None, 0.0, wg, nt)
                else:
                    args = (kind, c, a, b if kind == "triad" else None, 3.0, wg, nt)
                kpm.stream_kernel(*args)
                ts = []
                for _ in range(reps):
                    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
                    ev[0].record()
                    kpm.stream_kernel(*args)
                    ev[1].record()
                    torch.cuda.synchronize()
                    ts.append(ev[0].elapsed_time(ev[1]) * 1e-3)
                gbs = traffic / min(ts) / 1e9
                out["points"].append({"kind": kind, "wg_per_cu": wg, "nontemporal": nt, "GBps": round(gbs, 1)})
                if gbs > best.get(kind, {"GBps": 0.0})["GBps"]:
                    best[kind] = {"GBps": round(gbs, 1), "wg_per_cu": wg, "nontemporal": nt}
                if kind == "read" and float(part.sum().item()) != float(n):
                    raise RuntimeError("STREAM read kernel summed wrong values")
        if kind != "read":
            expect = 1.0 if kind == "copy" else 7.0
            if not bool(torch.all(c == expect).item()):
                raise RuntimeError(f"STREAM {kind} kernel wrote wrong values")
    for k in ("read", "copy", "triad"):
        out[k] = best[k]
    out["b_GBps"] = max(best[k]["GBps"] for k in ("read", "copy", "triad"))
    out["b_copy_GBps"] = best["copy"]["GBps"]
    del a, b, c, part
    return out


def leg_small(reps: int = 50):
    """The small correctness workload timed: 8 x 8 x 8 lattice (N = 2048), gamma = 1, R = 1, M = 128,
    complex128 (64 sweeps, launch-bound): kpm_moments launched op by op against its launch sequence
    captured once in a HIP graph and replayed."""
    import numpy as np
    import torch
    from paper_1410_5242_amd import inputs, kpm
    L, R, M = (8, 8, 8), 1, 128
    H = kpm.build_hamiltonian(L, inputs.potential(L, 1.0, 0))
    V0 = torch.from_numpy(inputs.phase_block(H.N, R, 0)).cuda()
    mu_e = kpm.moments(H, V0, M, check=False).cpu().numpy()
    mu = torch.empty((R, M), dtype=torch.float64, device="cuda")
    kpm.moments(H, V0, M, mu=mu, check=False, graph=True)
    torch.cuda.synchronize()
    same = bool(np.array_equal(mu.cpu().numpy(), mu_e))
    out = {"workload": f"TI 8x8x8 periodic (N={H.N}), gamma=1, R={R}, M={M}, complex128; {reps} back-to-back calls, "
                       "device-resident mu, one synchronisation at the end", "graph_equals_eager": same,
           "sweep_kernel": kpm.sweep_kernel(H, R)}
    for name, graph in (("eager", False), ("graph", True)):
        for _ in range(3):
            kpm.moments(H, V0, M, mu=mu, check=False, graph=graph)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            kpm.moments(H, V0, M, mu=mu, check=False, graph=graph)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        out[name] = {"us_per_call": round(dt * 1e6, 1), "us_per_sweep": round(dt * 1e6 / (M // 2), 2)}
    out["graph_speedup"] = round(out["eager"]["us_per_call"] / out["graph"]["us_per_call"], 2)
    H.close()
    return out


BATCH_TUNING_OVERRIDE = None   # (waves, wg_per_cu, dynamic, slab) from --batch-tuning


def leg_batched():
    """512 independent realisations, L in {12, 16, 20, 24}, gamma ~ U[0, 4], R = 8, M = 512, complex64:
    one persistent launch (graph replay), throughput over all instance sweeps."""
    import numpy as np
    import torch
    from paper_1410_5242_amd import autotune, inputs, kpm
    n, R, M = 512, 8, 512
    fam = inputs.instance_family(n, (12, 16, 20, 24), 4.0, 0)
    t0 = time.perf_counter()
    Hs = [kpm.build_hamiltonian(f["L"], inputs.potential(f["L"], f["gamma"], f["pot_seed"]), dtype="c64")
          for f in fam]
    V0s = [kpm.random_phase_block(H.N, R, f["vec_seed"], "c64") for f, H in zip(fam, Hs)]
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    cache = autotune.TuningCache()
    if BATCH_TUNING_OVERRIDE is not None:
        kpm.set_batch_tuning(*BATCH_TUNING_OVERRIDE)
        tuned = "override"
    else:
        tuned = autotune.apply_batched(cache, Hs, R)
    mu = kpm.moments_batched(Hs, V0s, M, graph=True)
    torch.cuda.synchronize()
    ts = []
    for _ in range(3):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        kpm.moments_batched(Hs, V0s, M, mu=mu, check=False, graph=True)
        ev[1].record()
        torch.cuda.synchronize()
        ts.append(ev[0].elapsed_time(ev[1]) / 1e3)
    t = min(ts)
    rows = sum(H.N for H in Hs)
    bps = sum(sweep_bytes(H.N, 13 * H.N, R, 8) for H in Hs)
    m = mu.cpu().numpy()
    out = {"workload": f"{n} instances, L in {{12,16,20,24}} (sum N = {rows}), gamma ~ U[0,4], R={R}, M={M}, "
                       f"complex64 + FP64 products, one persistent launch replayed from a HIP graph",
           "seconds": round(t, 4), "build_s": round(build_s, 2),
           "GBps": round(bps * (M // 2) / t / 1e9, 1), "pct_hbm_peak": round(100 * bps * (M // 2) / t / 1e9 / HBM_PEAK_GBS, 1),
           "gflops": round(sum(sweep_flops(H.N, R) for H in Hs) * (M // 2) / t / 1e9, 1),
           "bytes_per_all_instance_sweep": bps, "tuning": kpm.get_batch_tuning(), "autotuned": tuned,
           "mu0_max_dev": float(np.abs(m[:, :, 0] - 1.0).max())}
    kpm.reset_batch_tuning()
    for H in Hs:
        H.close()
    return out


def leg_variants(sweeps: int = 10):
    """Single fused sweeps on the 64^3 complex128 lattice for every block width R and the three
    variants (the paper's split of the sweep into plain SpMMV, the update without scalar
    products, and the full fused sweep): GB/s from the library's per-launch HIP events.  At
    R = 32 and 64 the index-reading sweeps run as well, forced by the tuning: the plain staged
    gather and its LDS-window variant."""
    import torch
    from paper_1410_5242_amd import autotune, inputs, kpm
    L = (64, 64, 64)
    H = kpm.build_hamiltonian(L, inputs.potential(L, 1.0, 0))
    N, Sd = H.N, 16
    out = {"workload": f"TI {L[0]}x{L[1]}x{L[2]} periodic, complex128, {sweeps} sweeps per point", "points": []}
    cache = autotune.TuningCache()
    for R, forced in [(R, None) for R in kpm.SUPPORTED_R] + [(R, g) for R in (32, 64) for g in (4, 3)]:
        kpm.reset_sweep_tuning()
        tuned = autotune.apply_sweep(cache, H, R, L)
        if forced is not None:
            # the index-reading sweeps at the widths the lattice sweep takes: the plain staged
            # gather (gather 4) in its best measured shape (two workgroups per CU, no die split,
            # natural row order) and its LDS-window variant (gather 3)
            t = kpm.get_sweep_tuning()
            t.update(lattice=0, gather=forced, wg_per_cu=2, xcd_ways=1, slab=0)
            kpm.set_sweep_tuning(**t)
            tuned = False
        V = kpm.random_phase_block(N, R, 1, "c128")
        W = kpm.random_phase_block(N, R, 2, "c128")
        eta = torch.zeros((2, R, 2), dtype=torch.float64, device="cuda")
        kernel = kpm.sweep_kernel(H, R)
        Si = 4   # the paper's model bytes for every kernel (the lattice sweep reads no indices)
        for var in ("full", "nodot", "plain"):
            e = eta if var == "full" else None
            kpm.aug_spmmv(H, V, W, 2.0 / H.a, -2.0 * H.b / H.a, -1.0, var, e)
            torch.cuda.synchronize()
            kpm.sweep_profile_read()
            kpm.sweep_profile_enable(True)
            for _ in range(sweeps):
                kpm.aug_spmmv(H, V, W, 2.0 / H.a, -2.0 * H.b / H.a, -1.0, var, e)
            torch.cuda.synchronize()
            kpm.sweep_profile_enable(False)
            n, tot, lo, hi = kpm.sweep_profile_read()
            avg_s = tot / n * 1e-3
            vec_streams = 2 if var == "plain" else 3
            byts = 13 * N * (Sd + Si) + vec_streams * R * Sd * N
            pt = {"R": R, "variant": var, "kernel": kernel, "avg_us": round(avg_s * 1e6, 1),
                  "GBps": round(byts / avg_s / 1e9, 1), "bytes": byts, "autotuned": tuned}
            if var == "full":
                pt["gflops"] = round(sweep_flops(N, R) / avg_s / 1e9, 1)
            out["points"].append(pt)
        del V, W
    kpm.reset_sweep_tuning()
    H.close()
    return out


def leg_sell(sweeps: int = 10):
    """The SELL-C-sigma path for general matrices (kpm_import_csr): single FULL sweeps at R = 1, 8
    and 32 from the library's per-launch HIP events, on two matrices handed over as host CRS: the
    64^3 complex128 lattice (the headline matrix, exported from the library's builder; 13 entries
    in every row, so no padding) and a seeded irregular Hermitian matrix of 2^20 rows (a power-law
    mix of row lengths, 2 % empty rows, half the couplings within 64 rows and half uniformly
    random); and the paper's 100 x 100 x 40 quantum-dot slab (open z, rows of 11 entries on its two
    surfaces) built straight into SELL storage by the lattice builder.  GB/s against the paper's
    model bytes Nnz (S_d + S_i) + 3 R S_d N, with Nnz the stored nonzeros without padding;
    stored/nnz is the layout's padding."""
    import torch
    from paper_1410_5242_amd import inputs, kpm
    L = (64, 64, 64)
    Hl = kpm.build_hamiltonian(L, inputs.potential(L, 1.0, 0))
    lattice = kpm.export_csr(Hl)
    Hl.close()
    irregular = inputs.random_hermitian_csr(1 << 20, seed=1)
    Ls = (100, 100, 40)
    slab_pot = inputs.quantum_dot_potential(Ls)
    out = {"workload": f"FULL sweeps, {sweeps} per point, complex128; matrices as host CRS, and the paper's "
                       f"100x100x40 quantum-dot slab (open z: its two surfaces have rows of 11 entries) built "
                       f"straight into SELL-C-sigma storage", "points": []}
    for name, csr, layouts in (
            ("TI 64x64x64 periodic", lattice, ((8, 1024), (1, 1), (32, 32))),
            ("irregular 2^20 rows", irregular, ((8, 1024), (1, 1), (32, 1), (32, 1024))),
            ("slab 100x100x40 quantum dots", None, ((8, 1024), (8, 1), (32, 1)))):
        for C, sigma in layouts:
            if csr is None:
                H = kpm.build_hamiltonian(Ls, slab_pot, periodic=(1, 1, 0), sell_C=C, sell_sigma=sigma)
                N, nnz = H.N, kpm.sell_info(H)["nnz"]
            else:
                rowptr, col, val = csr
                N, nnz = len(rowptr) - 1, int(rowptr[-1])
                H = kpm.import_csr(rowptr, col, val, C=C, sigma=sigma)
            stored = kpm.sell_info(H)["stored"]
            for R in (1, 8, 32):
                V = kpm.random_phase_block(N, R, 1, "c128")
                W = kpm.random_phase_block(N, R, 2, "c128")
                eta = torch.zeros((2, R, 2), dtype=torch.float64, device="cuda")
                kpm.aug_spmmv(H, V, W, 2.0 / H.a, -2.0 * H.b / H.a, -1.0, "full", eta)
                torch.cuda.synchronize()
                kpm.sweep_profile_read()
                kpm.sweep_profile_enable(True)
                for _ in range(sweeps):
                    kpm.aug_spmmv(H, V, W, 2.0 / H.a, -2.0 * H.b / H.a, -1.0, "full", eta)
                torch.cuda.synchronize()
                kpm.sweep_profile_enable(False)
                n, tot, lo, hi = kpm.sweep_profile_read()
                avg_s = tot / n * 1e-3
                byts = nnz * (16 + 4) + 3 * R * 16 * N
                out["points"].append({"matrix": name, "N": N, "nnz": nnz, "C": C, "sigma": sigma,
                                      "stored_over_nnz": round(stored / nnz, 3), "R": R,
                                      "kernel": kpm.sweep_kernel(H, R), "avg_us": round(avg_s * 1e6, 1),
                                      "GBps": round(byts / avg_s / 1e9, 1), "bytes": byts})
                del V, W
            H.close()
    return out


def leg_large(M: int = 200):
    """Blocks of 4 GiB or more, past one buffer descriptor's 32-bit offsets: the 128^3 lattice at
    R = 32 in complex128 (the lattice sweep addresses V, W and the matrix plane by plane) and the
    128 x 128 x 64 lattice at R = 64 (kpm_moments runs it as two 32-column groups).  Kernel time
    per sweep of the whole block from the library's HIP events over M/2 sweeps, GB/s of the model
    bytes Nnz (S_d + S_i) + 3 R S_d N of the whole block."""
    import torch
    from paper_1410_5242_amd import inputs, kpm
    out = {"workload": f"TI lattices gamma = 2 (seed 0), complex128, M = {M}, device random-phase blocks",
           "points": []}
    for L, R in (((128, 128, 128), 32), ((128, 128, 64), 64)):
        H = kpm.build_hamiltonian(L, inputs.potential(L, 2.0, 0))
        V0 = kpm.random_phase_block(H.N, R, 1, "c128")
        kpm.moments(H, V0, 8)
        torch.cuda.synchronize()
        kpm.sweep_profile_read()
        kpm.sweep_profile_enable(True)
        t0 = time.perf_counter()
        kpm.moments(H, V0, M)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        kpm.sweep_profile_enable(False)
        n, tot, lo, hi = kpm.sweep_profile_read()
        plan = kpm.sweep_plan(H, R)
        per_sweep_s = tot * 1e-3 / (M // 2)
        byts = sweep_bytes(H.N, 13 * H.N, R, 16)
        out["points"].append({"L": list(L), "R": R, "N": H.N, "block_GiB": round(H.N * R * 16 / 2 ** 30, 2),
                              "kernel": plan["kernel"], "group": plan["group"],
                              "ms_per_sweep": round(per_sweep_s * 1e3, 3),
                              "GBps": round(byts / per_sweep_s / 1e9, 1), "seconds": round(dt, 3)})
        del V0
        H.close()
        torch.cuda.empty_cache()
    return out


def leg_ladder(steps: int = 200, repeats: int = 3):
    """The paper's optimisation ladder on the 64^3 complex128 lattice, per start vector and KPM
    step (one moment pair): the naive algorithm (one SpMV and five BLAS-1 calls per step, one
    vector at a time), the fused sweep at R = 1 (the vector-at-a-time "throughput mode"), and
    the blocked fused sweep at R = 32.  Bytes per step and vector from the traffic model of
    Table "kpm_analysis" (naive) and of the fused algorithms, index bytes included."""
    import time
    import torch
    from paper_1410_5242_amd import autotune, inputs, kpm
    L = (64, 64, 64)
    H = kpm.build_hamiltonian(L, inputs.potential(L, 1.0, 0))
    N, Sd, nnz = H.N, 16, 13 * H.N
    M = 2 * steps
    cache = autotune.TuningCache()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        best = None
        for _ in range(repeats):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        return best

    out = {"workload": f"TI {L[0]}x{L[1]}x{L[2]} periodic, complex128, {steps} KPM steps per run, best of "
                       f"{repeats} runs; times per start vector and step", "stages": []}
    V1 = kpm.random_phase_block(N, 1, 1, "c128")
    kpm.reset_sweep_tuning()
    autotune.apply_sweep(cache, H, 1, L)
    t_naive = timed(lambda: kpm.moments_naive(H, V1, M, check=False)) / steps
    t_fused1 = timed(lambda: kpm.moments(H, V1, M, check=False)) / steps
    kern1 = kpm.sweep_kernel(H, 1)
    kpm.reset_sweep_tuning()
    R = 32
    autotune.apply_sweep(cache, H, R, L)
    VR = kpm.random_phase_block(N, R, 1, "c128")
    t_block = timed(lambda: kpm.moments(H, VR, M, check=False)) / steps / R
    kernR = kpm.sweep_kernel(H, R)
    kpm.reset_sweep_tuning()
    Si1 = SiR = 4   # the paper's model bytes (index bytes counted for every kernel)
    stages = [
        ("naive (SpMV + axpy, scal, axpy, nrm2, dot)", "R=1", t_naive, nnz * (Sd + 4) + 13 * N * Sd),
        ("fused sweep, one vector at a time", f"R=1, {kern1}", t_fused1, nnz * (Sd + Si1) + 3 * N * Sd),
        ("blocked fused sweep", f"R={R}, {kernR}", t_block, (nnz * (Sd + SiR) + 3 * R * N * Sd) / R),
    ]
    for name, shape, t, byts in stages:
        out["stages"].append({"stage": name, "shape": shape, "us_per_vector_step": round(t * 1e6, 2),
                              "model_bytes_per_vector_step": int(byts), "GBps": round(byts / t / 1e9, 1),
                              "speedup_vs_naive": round(t_naive / t, 2)})
    out["throughput_mode_penalty"] = round(t_fused1 / t_block, 2)
    del V1, VR
    H.close()
    return out


def leg_custom_roofline(sweeps: int = 20):
    """The paper's custom roofline P* = min(P*_MEM, P*_LLC) (eq. "eq:roofline_custom"): P*_LLC
    is measured on a down-sized problem whose whole working set (matrix and the three vector
    blocks) fits the 256 MB last-level cache, with the same kernel and launch shape as the
    full-size run; P*_MEM is the attainable HBM rate b over the model bytes (Omega = 1).
    Per block width R on 64 x 64 x Z lattices (complex128, Z chosen for about 130 MB), and for
    the batched solver on 256 instances of 8^3 sites (complex64, R = 8)."""
    import torch
    from paper_1410_5242_amd import autotune, inputs, kpm
    cache = autotune.TuningCache()
    out = {"workload": "complex128 TI lattices 64 x 64 x Z, Z = max(3, ~130 MB / (16384 rows x model bytes per "
                       "row)); sweeps timed with the library's per-launch HIP events", "points": []}
    for R in kpm.SUPPORTED_R:
        row_bytes = 13 * 20 + 3 * R * 16
        Z = max(3, int(round(130e6 / (16384 * row_bytes))))
        L = (64, 64, Z)
        H = kpm.build_hamiltonian(L, inputs.potential(L, 1.0, 0))
        kpm.reset_sweep_tuning()
        autotune.apply_sweep(cache, H, R, (64, 64, 64))   # the full-size run's launch shape
        V = kpm.random_phase_block(H.N, R, 1, "c128")
        W = kpm.random_phase_block(H.N, R, 2, "c128")
        eta = torch.zeros((2, R, 2), dtype=torch.float64, device="cuda")
        for _ in range(3):
            kpm.aug_spmmv(H, V, W, 2.0 / H.a, -2.0 * H.b / H.a, -1.0, "full", eta)
        torch.cuda.synchronize()
        kpm.sweep_profile_read()
        kpm.sweep_profile_enable(True)
        for _ in range(sweeps):
            kpm.aug_spmmv(H, V, W, 2.0 / H.a, -2.0 * H.b / H.a, -1.0, "full", eta)
        torch.cuda.synchronize()
        kpm.sweep_profile_enable(False)
        n, tot, lo, hi = kpm.sweep_profile_read()
        avg = tot / n * 1e-3
        byts = sweep_bytes(H.N, 13 * H.N, R, 16)
        out["points"].append({"R": R, "L": list(L), "working_set_MB": round(byts / 1e6, 1),
                              "kernel": kpm.sweep_kernel(H, R), "avg_us": round(avg * 1e6, 2),
                              "llc_GBps": round(byts / avg / 1e9, 1),
                              "llc_gflops": round(sweep_flops(H.N, R) / avg / 1e9, 1)})
        del V, W
        H.close()
        torch.cuda.empty_cache()
    kpm.reset_sweep_tuning()
    # batched solver: 256 instances of 8^3 sites, one per CU, all resident in the last-level cache
    n, Rb, M = 256, 8, 512
    fam = inputs.instance_family(n, (8,), 4.0, 0)
    Hs = [kpm.build_hamiltonian(f["L"], inputs.potential(f["L"], f["gamma"], f["pot_seed"]), dtype="c64")
          for f in fam]
    V0s = [kpm.random_phase_block(H.N, Rb, f["vec_seed"], "c64") for f, H in zip(fam, Hs)]
    if BATCH_TUNING_OVERRIDE is not None:
        kpm.set_batch_tuning(*BATCH_TUNING_OVERRIDE)
    else:
        autotune.apply_batched(cache, Hs, Rb)
    mu = kpm.moments_batched(Hs, V0s, M, graph=True)
    torch.cuda.synchronize()
    ts = []
    for _ in range(3):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        kpm.moments_batched(Hs, V0s, M, mu=mu, check=False, graph=True)
        ev[1].record()
        torch.cuda.synchronize()
        ts.append(ev[0].elapsed_time(ev[1]) / 1e3)
    t = min(ts)
    bps = sum(sweep_bytes(H.N, 13 * H.N, Rb, 8) for H in Hs)
    out["batched"] = {"workload": f"{n} instances of 8^3 sites (sum N = {sum(H.N for H in Hs)}), gamma ~ U[0,4], "
                                  f"R={Rb}, M={M}, complex64, one persistent launch",
                      "working_set_MB": round(bps / 1e6, 1), "seconds": round(t, 5),
                      "llc_GBps": round(bps * (M // 2) / t / 1e9, 1)}
    kpm.reset_batch_tuning()
    for H in Hs:
        H.close()
    return out


def leg_spectral(M: int = 1000, K: int = 1024):
    """Local DOS of 16 sites and A(k, E) at 16 momenta on the 64^3 complex128 lattice (gamma = 1):
    the fused blocked sweep on deterministic start vectors (4 orbitals x 16 = R = 64 per run),
    then the batched Jackson reconstruction."""
    import math
    import time
    import torch
    from paper_1410_5242_amd import autotune, inputs, kpm, spectral
    L = (64, 64, 64)
    H = kpm.build_hamiltonian(L, inputs.potential(L, 1.0, 0))
    kpm.reset_sweep_tuning()
    tuned = autotune.apply_sweep(autotune.TuningCache(), H, 64, L)
    E = torch.linspace(H.b - 0.999 * H.a, H.b + 0.999 * H.a, K, dtype=torch.float64, device="cuda")
    sites = [x + 64 * (y + 64 * 32) for x, y in ((4 * i, 3 * i) for i in range(16))]
    ks = [(math.pi * i / 15, 0.0, 0.0) for i in range(16)]   # Gamma -> X
    out = {"workload": f"TI 64x64x64 periodic, gamma=1, complex128, M={M}, {K} energies; 16 sites / 16 momenta, "
                       "4 orbitals each (R = 64 per run)", "kernel": kpm.sweep_kernel(H, 64), "autotuned": tuned}
    Sd, N = 16, H.N
    bps = 13 * N * Sd + 3 * 64 * N * Sd
    for name, fn in (("local_dos", lambda: spectral.local_dos(H, L, sites, M, E)),
                     ("spectral_function", lambda: spectral.spectral_function(H, L, ks, M, E))):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, rho = fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        integ = float((rho.sum(dim=1) * (E[1] - E[0])).mean().item())
        out[name] = {"seconds": round(dt, 4), "GBps": round(bps * (M // 2) / dt / 1e9, 1),
                     "mean_integral": round(integ, 4)}
    kpm.reset_sweep_tuning()
    H.close()
    return out


def leg_slab(M: int = 2000, R: int = 32):
    """The paper's own geometry: slabs of 100 x 100 x 40 (its performance-model domain) and
    200 x 100 x 40 sites (its single-device domain), periodic in x and y, open in z, with a
    superlattice of quantum dots in the top layers; complex128, R = 32, M = 2000, Jackson DOS."""
    import torch
    from paper_1410_5242_amd import autotune, inputs, kpm
    out = {"workload": f"TI slabs periodic in x, y, open in z; quantum dots (period 25, radius 6, 4 layers, "
                       f"V = 1) + disorder gamma = 0.2; complex128, R = {R}, M = {M}", "points": []}
    for L in ((100, 100, 40), (200, 100, 40)):
        pot = inputs.quantum_dot_potential(L)
        H = kpm.build_hamiltonian(L, pot, periodic=(1, 1, 0))
        kpm.reset_sweep_tuning()
        tuned = autotune.apply_sweep(autotune.TuningCache(), H, R, L)
        V0 = kpm.random_phase_block(H.N, R, 1, "c128")
        kpm.moments(H, V0, 8)
        torch.cuda.synchronize()
        kpm.sweep_profile_read()
        kpm.sweep_profile_enable(PROFILE_PERIOD)
        t0 = time.perf_counter()
        mu = kpm.moments(H, V0, M)
        E = torch.linspace(H.b - 0.999 * H.a, H.b + 0.999 * H.a, 4096, dtype=torch.float64, device="cuda")
        rho = kpm.dos(mu, H.a, H.b, E)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        kpm.sweep_profile_enable(False)
        n, tot, lo, hi = kpm.sweep_profile_read()
        kernel = kpm.sweep_kernel(H, R)
        Si = 0 if kernel == "lattice_kernel" else 4
        N = H.N
        nnz = 13 * N - 2 * 2 * 4 * L[0] * L[1]   # the two surfaces lack their outward z neighbour
        stored = 13 * N * (16 + Si) + 3 * R * 16 * N
        model = nnz * (16 + 4) + 3 * R * 16 * N
        avg = tot / max(n, 1) * 1e-3
        out["points"].append({"L": list(L), "N": N, "kernel": kernel, "autotuned": tuned,
                              "seconds": round(dt, 4), "sweep_avg_us": round(avg * 1e6, 1),
                              "GBps_stored": round(stored / avg / 1e9, 1),
                              "GBps_paper_model": round(model / avg / 1e9, 1),
                              "gflops": round(sweep_flops(N, R) / avg / 1e9, 1),
                              "dos_integral": round(float(rho.sum().item() * (E[1] - E[0]).item()), 4)})
        kpm.reset_sweep_tuning()
        H.close()
        del V0, mu
    return out


def leg_bounds():
    """Spectral bounds on the 64^3 complex128 lattice (gamma = 1): Gershgorin discs (fused into
    the build) against the extreme Ritz values of 25, 50 and 100 Lanczos steps on the device.
    A tighter half-width a gives proportionally finer energy resolution per moment."""
    import time
    import torch
    from paper_1410_5242_amd import inputs, kpm
    L = (64, 64, 64)
    H = kpm.build_hamiltonian(L, inputs.potential(L, 1.0, 0))
    a_g = (H.emax - H.emin) / 2
    out = {"workload": "TI 64x64x64 periodic, gamma=1, complex128",
           "gershgorin": {"emin": round(H.emin, 6), "emax": round(H.emax, 6)}, "lanczos": []}
    kpm.lanczos_bounds(H, 4, 1)
    for steps in (25, 50, 100):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lo, hi = kpm.lanczos_bounds(H, steps, 1)
        dt = time.perf_counter() - t0
        out["lanczos"].append({"steps": steps, "emin": round(lo, 6), "emax": round(hi, 6),
                               "seconds": round(dt, 4), "halfwidth_ratio_vs_gershgorin": round(((hi - lo) / 2) / a_g, 4)})
    # resolution per moment: DOS L1 error against the finest Lanczos-scaled DOS (M = 4096), on a
    # common energy grid, for moment prefixes of one M = 4096 run per scaling (R = 32 vectors)
    R, Mmax, K = 32, 4096, 2048
    a_l, b_l = 1.01 * (hi - lo) / 2, (hi + lo) / 2
    V0 = kpm.random_phase_block(H.N, R, 3, "c128")
    E = torch.linspace(lo, hi, K, dtype=torch.float64, device="cuda")
    dE = float(E[1] - E[0])
    mus = {}
    for name, (a, b) in (("gershgorin", (H.a, H.b)), ("lanczos", (a_l, b_l))):
        kpm.set_scaling(H, a, b)
        mus[name] = (kpm.moments(H, V0, Mmax), a, b)
    ref = kpm.dos(*mus["lanczos"][:1], mus["lanczos"][1], mus["lanczos"][2], E)
    curve = {"gershgorin": {}, "lanczos": {}}
    for name, (mu, a, b) in mus.items():
        for M in (64, 128, 256, 512, 1024, 2048):
            rho = kpm.dos(mu[:, :M].contiguous(), a, b, E)
            curve[name][M] = round(float((rho - ref).abs().sum().item() * dE), 5)
    need = {}
    for eps in (0.05, 0.02):
        need[str(eps)] = {n: next((M for M, l1 in sorted(c.items()) if l1 <= eps), None) for n, c in curve.items()}
    out["resolution"] = {"workload": f"R = {R}, reference: Lanczos scaling (100 steps, 1.01 margin) at M = {Mmax}; "
                                     f"{K} energies on the Lanczos interval; L1 = sum |rho - ref| dE",
                         "l1_vs_M": curve, "M_needed": need}
    del V0
    H.close()
    return out


def leg_time_to_dos():
    from paper_1410_5242_amd import learned, time_to_dos
    if not os.path.exists(learned.WEIGHTS):
        return {"skipped": "no trained network weights at " + os.path.relpath(learned.WEIGHTS, ROOT)}
    return time_to_dos.run(log=log)


COPY_BYTES = 1 << 30


def probe(args, H, V0, M, R, Sd):
    """Calibration kernels of known traffic plus a few sweeps, for rocprofv3 --pmc runs: the
    library's STREAM read (reads COPY_BYTES) and copy (reads and writes COPY_BYTES) kernels, then
    --probe-sweeps fused sweeps of the workload."""
    import torch
    from paper_1410_5242_amd import kpm
    a = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=V0.device)
    c = torch.empty_like(a)
    cus = torch.cuda.get_device_properties(V0.device).multi_processor_count
    part = torch.zeros(cus, dtype=torch.float64, device=V0.device)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    kpm.stream_kernel("read", part, a, wg_per_cu=1, nontemporal=True)
    ev[1].record()
    kpm.stream_kernel("copy", c, a, wg_per_cu=1, nontemporal=True)
    ev[2].record()
    torch.cuda.synchronize()
    read_ms, copy_ms = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    del a, c
    kpm.sweep_profile_read()
    kpm.sweep_profile_enable(True)
    mu = kpm.moments(H, V0, 2 * args.probe_sweeps)
    torch.cuda.synchronize()
    kpm.sweep_profile_enable(False)
    n, tot, lo, hi = kpm.sweep_profile_read()
    bps = sweep_bytes(H.N, 13 * H.N, R, Sd)
    print(json.dumps({"probe": True, "calibration_bytes": COPY_BYTES, "read_ms": round(read_ms, 4),
                      "copy_ms": round(copy_ms, 4), "sweeps": n, "sweep_avg_ms": round(tot / max(n, 1), 5),
                      "sweep_algorithmic_bytes": bps, "mu0": float(mu[0, 0].item())}), flush=True)
    H.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ti64_r32_m2000_c128", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-target-s", type=float, default=15.0)
    ap.add_argument("--probe", action="store_true",
                    help="short run for hardware counters: the STREAM read and copy kernels over 1 GiB "
                         "(calibration kernels of known traffic) and --probe-sweeps fused sweeps of the workload")
    ap.add_argument("--probe-sweeps", type=int, default=8)
    ap.add_argument("--batch-tuning", default=None,
                    help="waves,wg_per_cu,dynamic,slab for the batched leg instead of the tuning cache")
    ap.add_argument("--legs", default="small,variants,custom_roofline,ladder,precision,batched,spectral,slab,bounds,"
                                      "sell,large,time_to_dos,oracle_subsets",
                    help="extra measurements after the headline step (comma separated): any of small, variants, "
                         "custom_roofline, ladder, precision, batched, spectral, slab, bounds, sell, large, "
                         "time_to_dos, oracle_subsets; or none")
    args = ap.parse_args()
    if args.batch_tuning:
        global BATCH_TUNING_OVERRIDE
        BATCH_TUNING_OVERRIDE = tuple(int(v) for v in args.batch_tuning.split(","))
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU sharding is a design, "
              f"not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1410_5242_amd import autotune, inputs, kpm

    L, gamma, R, M, dtype, K = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"[bench] workload {args.workload}: L={L} gamma={gamma} R={R} M={M} dtype={dtype}")

    pot = inputs.potential(L, gamma, 0)
    t0 = time.perf_counter()
    H = kpm.build_hamiltonian(L, pot, dtype=dtype)
    build_s = time.perf_counter() - t0
    N = H.N
    Sd = 16 if dtype == "c128" else 8
    V0 = torch.from_numpy(inputs.phase_block(N, R, 0, dtype=np.complex128 if dtype == "c128" else np.complex64)).to(dev)
    E = torch.from_numpy((H.b + H.a * (-1.0 + (2.0 * np.arange(K) + 1.0) / K))).to(dev)
    mu = torch.empty((R, M), dtype=torch.float64, device=dev)
    rho = torch.empty(K, dtype=torch.float64, device=dev)
    # launch shape from the committed autotuner cache, if it holds this workload
    autotuned = autotune.apply_sweep(autotune.TuningCache(), H, R, L)
    sweep_kernel = kpm.sweep_kernel(H, R)
    log(f"[bench] built H: N={N} a={H.a:.6f} b={H.b:.6f} ({build_s:.3f} s); sweep kernel {sweep_kernel}")

    if args.probe:
        probe(args, H, V0, M, R, Sd)
        return

    def step():
        kpm.moments(H, V0, M, mu=mu, check=True)
        kpm.dos(mu, H.a, H.b, E, kernel="jackson", rho=rho)

    for i in range(args.warmup):
        step()
        log(f"[bench] warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()

    kpm.sweep_profile_read()                 # clear
    # time every PROFILE_PERIOD-th sweep kernel: each event pair costs a few
    # microseconds of stream time, so timing all 1000 sweeps of a step would
    # slow the step it measures by about 2 %
    kpm.sweep_profile_enable(PROFILE_PERIOD)
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for i in range(args.steps):
        step()
        log(f"[bench] step {i + 1}/{args.steps} done")
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kpm.sweep_profile_enable(False)
    n_sweeps, sweep_ms_tot, sweep_ms_min, sweep_ms_max = kpm.sweep_profile_read()
    ms_per_step = ev0.elapsed_time(ev1) / args.steps

    sweeps_per_step = M // 2
    nnz = 13 * N
    # algorithmic bytes: the paper's minimum traffic of the blocked sweep with CRS / SELL
    # storage, Nnz (S_d + S_i) + 3 R S_d N; the lattice kernel reads no column indices, so the
    # bytes it must move are the same with S_i = 0 (reported beside it)
    bps = sweep_bytes(N, nnz, R, Sd, 4)
    bps_stored = sweep_bytes(N, nnz, R, Sd, 0 if sweep_kernel == "lattice_kernel" else 4)
    fps = sweep_flops(N, R)
    value = bps * sweeps_per_step / (ms_per_step * 1e-3) / 1e9
    gflops = fps * sweeps_per_step / (ms_per_step * 1e-3) / 1e9
    sweep_avg_ms = sweep_ms_tot / max(1, n_sweeps)
    achieved = bps / (sweep_avg_ms * 1e-3) / 1e9
    rho_h = rho.cpu().numpy()
    dos_integral = float(rho_h.sum() * 2.0 * H.a / K)

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if dtype == "c128" else "f32 (f64 products)",
        "data": "synthetic",
        "config": {
            "workload": f"KPM-DOS, TI Hamiltonian {L[0]}x{L[1]}x{L[2]} periodic (N={N}, 13 nnz/row), "
                        f"gamma={gamma}, R={R}, M={M}, {dtype}, Jackson DOS on {K} energies",
            "sweeps_per_step": sweeps_per_step,
            "bytes_per_sweep": bps,
            "bytes_per_sweep_kernel_minimum": bps_stored,
            "flops_per_sweep": fps,
        },
        "pct_hbm_peak": round(100.0 * value / HBM_PEAK_GBS, 2),
        "gflops": round(gflops, 1),
        "time_to_moments_and_dos_ms": round(ms_per_step, 3),
        "dos_integral": round(dos_integral, 8),
        "wall_s": round(wall, 3),
        "build_ms": round(build_s * 1e3, 1),
        "roofline": {
            "bound": "hbm",
            "kernel": sweep_kernel,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_record(sweep_kernel, args.workload),
            "launches": n_sweeps,
            "launches_timed_every": PROFILE_PERIOD,
            "avg_launch_ms": round(sweep_avg_ms, 5),
            "min_launch_ms": round(sweep_ms_min, 5),
            "max_launch_ms": round(sweep_ms_max, 5),
            "algorithmic_bytes_per_launch": bps,
        },
        "tuning": {"autotuned": autotuned, "sweep": kpm.get_sweep_tuning()},
    }
    kpm.reset_sweep_tuning()
    H.close()
    del V0
    log("[bench] attainable bandwidth (STREAM copy / triad)")
    out["stream"] = leg_stream()
    torch.cuda.empty_cache()
    b_meas = out["stream"]["b_GBps"]
    out["roofline"]["measured_b_GBps"] = b_meas
    out["roofline"]["frac_of_measured_b"] = round(achieved / b_meas, 4)
    out["roofline"]["measured_b_copy_GBps"] = out["stream"]["b_copy_GBps"]
    out["pct_of_measured_b"] = round(100.0 * value / b_meas, 2)
    legs = [x for x in args.legs.split(",") if x and x != "none"]
    for name, fn in (("small", leg_small), ("variants", leg_variants), ("custom_roofline", leg_custom_roofline),
                     ("ladder", leg_ladder),
                     ("precision", leg_precision), ("batched", leg_batched), ("spectral", leg_spectral),
                     ("slab", leg_slab), ("bounds", leg_bounds), ("sell", leg_sell), ("large", leg_large),
                     ("time_to_dos", leg_time_to_dos)):
        if name in legs:
            log(f"[bench] leg {name}")
            out[name] = fn()
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
    # custom roofline: P* = min(b, P*_LLC) per R against the full-size measurement of the same kernel
    if "custom_roofline" in out and "variants" in out:
        full = {(p["R"], p["kernel"]): p for p in out["variants"]["points"] if p["variant"] == "full"}
        for p in out["custom_roofline"]["points"]:
            q = full.get((p["R"], p["kernel"]))
            p["mem_bound_GBps"] = b_meas
            p["p_star_GBps"] = round(min(b_meas, p["llc_GBps"]), 1)
            if q:
                p["full_size_GBps"] = q["GBps"]
                p["full_size_frac_of_p_star"] = round(q["GBps"] / p["p_star_GBps"], 3)
        if "batched" in out:
            cb = out["custom_roofline"]["batched"]
            cb["mem_bound_GBps"] = b_meas
            cb["p_star_GBps"] = round(min(b_meas, cb["llc_GBps"]), 1)
            cb["family512_GBps"] = out["batched"]["GBps"]
            cb["family512_frac_of_p_star"] = round(out["batched"]["GBps"] / cb["p_star_GBps"], 3)
    # fractions of the measured bandwidth b beside those of the 8 TB/s peak
    for rec in [out.get("precision", {}).get(d, {}) for d in ("c128", "c64")] + [out.get("batched", {})] + \
            out.get("slab", {}).get("points", []):
        for key in ("GBps", "GBps_paper_model"):
            if key in rec:
                rec[f"pct_of_measured_b{key[4:]}"] = round(100.0 * rec[key] / b_meas, 1)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(L, gamma, R, dtype, args.cpu_target_s)
        if "oracle_subsets" in legs:
            log("[bench] oracle on subsets of the other workloads")
            out["cpu_baseline"]["subsets"] = cpu_oracle_subsets()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
