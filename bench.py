#!/usr/bin/env python3
"""Benchmark of the fused fluctuating D2Q9 step (f-norm basis) on one GPU.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload large|ensemble|serve|paper|d3q19|config2|cpu]

Default workload ("large"): one 8192 x 8192 periodic lattice, FP32 storage
shifted by f^0(rho0, u0), rho0 = 1, u_x0 = 0.1, kT = 1e-4, all tau = 1, initial
transverse shear wave u_y = 1e-3 sin(2 pi x / L).  One step is the whole
hot path: the fused collide-and-stream kernel over all sites; every 100
steps the structure factor of rho, j~_x, j~_y is sampled (2-D FFT) and the
shear-mode amplitude j~_y(k = 2 pi / L) is read back.  Before the W warm-up
steps the run measures two bandwidth probes (the step's loads and stores
without arithmetic, and a contiguous copy of the same bytes), picks the
launch shape (unless --launch fixes it) and steps a second lattice of the
same shape for ~0.3 s, untimed, so that the timed steps start at the clock
the board's power limit settles the step at.

Prints one JSON line: MLUPS (lattice-site updates per second / 1e6) over
the timed steps, the step kernel's achieved HBM bandwidth against the
8 TB/s peak (72 algorithmic bytes per site update: nine FP32 reads and nine
FP32 writes in place), a served-requests measurement (solves/s and p50/p99
latency of mixed Poisson-arriving requests through the continuous-batching
server, next to the plain FP64 one-lattice-per-launch path on the same
arrivals), and the FP64 CPU oracle's rate on a bounded sample of the
large workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_SITE = {"f32": 72, "f64": 144}
# D3Q19 FP32 f-norm step: VALU wavefront instructions per wavefront (= per
# site), SQ_INSTS_VALU / SQ_WAVES averaged over both phases,
# profiles/step3_fp32_256cube_d3q19.md
D3Q19_VALU_PER_SITE = 2095
# FP32 floating-point operations per site of that kernel (its variant for
# one relaxation time, which this workload's tau = 1 selects), counted in its
# gfx950 code: FMAs 2 each (1519 v_fma/v_fmac/v_fmamk), multiplies, adds and
# subtracts 1 each (225 + 85), transcendentals (rsq, rcp, sqrt, log, sin,
# cos) 1 each (48); conversions, compares and min/max are not counted.  One
# lane computes one site.
D3Q19_FLOPS_PER_SITE = 3396
# the same for the FP64 kernel of that workload: 1804 FMAs, 327 multiplies,
# 117 adds and subtracts, 33 transcendentals (FP64 operations)
D3Q19_FP64_FLOPS_PER_SITE = 4085
# FP32 vector peak without packed (two-wide) instructions, which this
# library does not use: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz;
# the FP64 vector peak is the same
FP32_VECTOR_PEAK = 256 * 4 * 16 * 2 * 2.4e9
FP64_VECTOR_PEAK = FP32_VECTOR_PEAK
# VALU issue peak: 256 CUs x 4 SIMDs, one wavefront instruction (64 lanes,
# 16 per cycle) every 4 cycles at 2.4 GHz
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4
# sources of the step kernel (the one whose HBM traffic the profiles record)
KERNEL_SOURCES = ["paper_1204_6734_amd/csrc/flb_device.hpp",
                  "paper_1204_6734_amd/csrc/fp64_series.hpp",
                  "paper_1204_6734_amd/csrc/flb_buffer.hpp",
                  "paper_1204_6734_amd/csrc/flb_step.hip",
                  "paper_1204_6734_amd/csrc/flb_kernels.hpp"]


def kernel_hash() -> str:
    """Hash of the step kernel's sources with comments and blank space
    taken out, so that a change of wording leaves the counter record valid
    and any change of code does not."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def traffic_from_profiles(name: str):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{name}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_hash") != kernel_hash():
        return None
    return d.get("bytes_per_launch")


# --basis of the large workload: (config name, basis code of the C ABI)
BASES = {"fnorm": ("fnorm_local", 0), "hermite": ("hermite", 1), "lut": ("fnorm_lut", 2)}


def host_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_rate(nx: int, ny: int, threads: int, seconds: float = 0.0, steps: int = 0,
                **kw) -> dict:
    """MLUPS of the FP64 oracle on an nx x ny lattice with `threads` threads,
    for `steps` steps or until ~`seconds` have passed (chunks of 20)."""
    import oracle as O
    O.set_threads(threads)
    try:
        L = O.Lattice(O.make_params(nx, ny, **kw))
        L.step(2)
        done, t0 = 0, time.perf_counter()
        while (steps and done < steps) or (not steps and time.perf_counter() - t0 < seconds):
            k = min(20, steps - done) if steps else 20
            L.step(k)
            done += k
        dt = time.perf_counter() - t0
        L.close()
    finally:
        O.set_threads(1)
    return {"mlups": nx * ny * done / dt / 1e6, "steps": done, "seconds": round(dt, 2),
            "threads": threads}


def cpu_baseline(seconds: float = 12.0, basis: int = 0, ux0: float = 0.1) -> dict:
    """FP64 oracle on a bounded sample of the large workload (a 128 x 128
    lattice with its parameters and basis): a third of ~`seconds` on one
    thread, the rest on every host core (the oracle's per-site loops in
    OpenMP threads)."""
    nx = ny = 128
    kw = dict(rho0=1.0, ux0=ux0, kT=1e-4, seed=1, basis=basis)
    cores = host_cores()
    one = oracle_rate(nx, ny, 1, seconds=seconds / 3, **kw)
    allc = oracle_rate(nx, ny, cores, seconds=2 * seconds / 3, **kw)
    return {"value": allc["mlups"], "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{nx}x{ny} lattice, same parameters as the timed workload, FP64 C "
                      f"oracle: {allc['steps']} steps on {cores} threads in "
                      f"{allc['seconds']} s; {one['steps']} steps on 1 thread in "
                      f"{one['seconds']} s", "single_thread_mlups": one["mlups"],
            "cpu_model": cpu_model()}


def cpu_plan() -> dict:
    """The oracle timings of the statistics workloads, one thread and every
    core: 32 x 32 at rest for 1e4 steps sampling every step, and 1e3 steps
    of the 256 x 256 mixed-tau workload per u_x0 in {0, 0.1, 0.2}."""
    from paper_1204_6734_amd import inputs as I
    cores = host_cores()
    out = {"cores": cores, "cpu_model": cpu_model()}
    for threads in (1, cores):
        r = oracle_rate(32, 32, threads, steps=10000, kT=1e-4, seed=1, sample_every=1,
                        block_steps=500)
        out[f"32x32_rest_1e4_steps_{threads}t"] = r
        print(f"cpu plan: 32x32 on {threads} threads: {r['mlups']:.2f} MLUPS",
              file=sys.stderr, flush=True)
        for u in (0.0, 0.1, 0.2):
            r = oracle_rate(256, 256, threads, steps=1000, ux0=u, kT=1e-4,
                            tau=I.mixed_taus(2), seed=1, sample_every=1, block_steps=500)
            out[f"256x256_mixed_tau_u{u:g}_1e3_steps_{threads}t"] = r
            print(f"cpu plan: 256x256 u0={u} on {threads} threads: {r['mlups']:.2f} MLUPS",
                  file=sys.stderr, flush=True)
    return out


def run_large(F, torch, steps: int, warmup: int, nx: int = 8192, every: int = 100,
              launch=None, basis: str = "fnorm", precision: str = "fp32", ux0: float = 0.1,
              sample_every: int = 0):
    from paper_1204_6734_amd import inputs as I
    stream = torch.cuda.current_stream()
    bname, bcode = BASES[basis]
    fp32 = precision == "fp32"
    p = F.make_params(nx, nx, precision=F.FP32_SHIFTED if fp32 else F.FP64, basis=bcode,
                      rho0=1.0, ux0=ux0, kT=1e-4, seed=1, init=F.INIT_FIELDS, sk_every=every,
                      sample_every=sample_every, block_steps=100 if sample_every > 0 else 0)
    L = F.Lattice(p, stream=stream)
    L.set_fields(*I.shear_wave_fields(nx, nx, ux0=ux0, amp=1e-3))
    # the two bandwidth probes (the step's access pattern without arithmetic,
    # and a plain contiguous copy of the same bytes) run first
    bps = BYTES_PER_SITE["f32" if fp32 else "f64"]
    probes = {"copy_ms": F.copy_probe(nx, nx, F.FP32_SHIFTED if fp32 else F.FP64, reps=20),
              "stream_bytes": bps // 2 * nx * nx}
    probes["stream_ms"] = F.stream_copy_probe(probes["stream_bytes"], reps=20)
    if launch is None:
        tune = L.autotune(reps=3)  # trial steps run on a copy of the state
    else:
        L.set_launch(*launch)
        tune = "fixed by --launch"

    chunk = every if every > 0 else 100
    # The step runs at the board's power limit (1400 W): after the lighter
    # work above (the probes, and launch trials with host synchronisations
    # between them) the shader clock needs tens of milliseconds of
    # continuous steps to settle at the step's own level, longer than a few
    # warm-up steps.  A second lattice of the same shape and launch shape
    # steps for ~0.3 s right before the warm-up, in the same stream; it is
    # untimed and shares nothing with the timed lattice, whose own warm-up is
    # the W steps below.
    settle = F.Lattice(F.make_params(nx, nx, precision=p.precision, basis=bcode, rho0=1.0,
                                     ux0=ux0, kT=1e-4, seed=2, sample_every=sample_every,
                                     block_steps=p.block_steps), stream=stream)
    lc = L.get_launch()
    settle.set_launch(lc["tiles_per_block"], lc["grid_blocks"])
    settle_steps = min(20000, max(20, int(round(300.0 / probes["copy_ms"]))))

    def run(n):
        done = 0
        log = []
        while done < n:
            k = min(chunk, n - done)
            L.step(k)
            done += k
            if every > 0 and done % every == 0:
                log.append(L.fourier_mode(2, 1, 0))
        return log

    settle.step(settle_steps)
    run(warmup)
    L.sync()
    torch.cuda.synchronize()
    settle.close()
    L.profile(True)
    L.kernel_time()  # reset
    tw0 = L.t
    t0 = time.perf_counter()
    log = run(steps)
    L.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kms, launches = L.kernel_time()
    L.profile(False)
    sites = nx * nx
    # structure-factor samples and mode logs that fell in the timed steps
    n_sk = (len([t for t in range(tw0, tw0 + steps) if t % every == 0]) if every > 0 else 0)
    with_sk = None
    if every > 0:
        # one window of `every` steps holding exactly one S(k) sample and one
        # mode readback: the rate of the whole workload at its own ratio
        ahead = (every - L.t % every) % every
        if ahead:
            L.step(ahead)
        L.sync()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L.step(every)  # samples S(k) at its first step
        L.fourier_mode(2, 1, 0)
        torch.cuda.synchronize()
        dt1 = time.perf_counter() - t1
        with_sk = {"steps": every, "sk_samples": 1, "mode_logs": 1,
                   "ms_per_step": round(dt1 * 1e3 / every, 4),
                   "mlups": round(sites * every / dt1 / 1e6, 1)}
    return {"sites": sites, "dt": dt, "kernel_ms": kms / max(launches, 1), "launches": launches,
            "mode_log": [abs(z) for z in log[-3:]], "probes": probes, "settle_steps": settle_steps,
            "sk_in_window": n_sk, "mode_logs_in_window": len(log), "with_sk": with_sk,
            "launch": {"chosen": L.get_launch(), "candidates": tune},
            "config": {"workload": f"{nx}x{nx} D2Q9 {'FP32-shifted' if fp32 else 'FP64'}, "
                                   f"{'' if basis == 'fnorm' else bname + ' basis, '}"
                                   f"rho0=1, u_x0={ux0:g}, kT=1e-4, "
                                   f"tau=1, shear wave 1e-3 sin(2 pi x/L); " +
                                   (f"S(k) and j~_y(2 pi/L) every {every} steps "
                                    f"({n_sk} S(k) samples and {len(log)} mode logs in the "
                                    f"{steps} timed steps; 'with_sk' times {every} steps "
                                    f"holding one of each)" if every > 0
                                    else "no S(k), no mode log") +
                                   (f"; correlators every {sample_every} steps"
                                    if sample_every > 0 else ""),
                       "nx": nx, "ny": nx, "precision": "fp32_shifted" if fp32 else "fp64",
                       "basis": bname, "sk_every": every, "sample_every": sample_every,
                       "parallelism": "single GPU"},
            "dtype": "f32" if fp32 else "f64",
            # FP32 storage computes the collision in FP64 above |u0| = 0.25
            "kernel_label": "step_kernel<%s,%s>" % (
                ("float,float" if abs(ux0) <= 0.25 else "float,double") if fp32
                else "double,double", bname) +
                (f" (correlator-sampling variant every {sample_every} steps)"
                 if sample_every > 0 else ""),
            "kernel_name": f"step_{precision}_{nx}" + ("" if basis == "fnorm" else f"_{basis}") +
                           ("_fp64compute" if fp32 and abs(ux0) > 0.25 else "") +
                           (f"_sample{sample_every}" if sample_every > 0 else "")}


def run_ensemble(F, torch, steps: int, warmup: int, n: int = 64, side: int = 128,
                 chunk: int = 100, every: int = 10):
    """64 replicas of 128 x 128 in one batched launch per step, replayed from
    a captured hipGraph of `chunk` steps; correlators every `every` steps."""
    from paper_1204_6734_amd import inputs as I
    ps = [F.make_params(side, side, precision=F.FP32_SHIFTED, ux0=m["ux0"], kT=m["kT"],
                        seed=m["seed"], sample_every=every, block_steps=100)
          for m in I.ensemble_members(n, seed=3)]
    E = F.Ensemble(ps, stream=torch.cuda.current_stream(), graph_chunk=chunk)
    tune = E.autotune(reps=5)
    E.step(warmup)
    E.sync()
    t0 = time.perf_counter()
    E.step(steps)
    E.sync()
    dt = time.perf_counter() - t0
    c = E.covariance(0)
    return {"mlups": n * side * side * steps / dt / 1e6, "seconds": dt, "replicas": n,
            "side": side, "steps": steps, "graph_chunk": chunk, "sample_every": every,
            "replica0_nsamples": c["nsamples"],
            "launch": {"chosen": E.get_launch(), "candidates": tune}}


def run_serving(F, torch, nreq: int = 40, rate: float = 50.0, chunk: int = 100,
                every: int = 10, baseline: bool = True):
    """Poisson arrivals of mixed requests (side log-uniform 64..2048, steps
    log-uniform 1e3..1e5, kT log-uniform 1e-5..1e-3, u_x0 ~ U[0, 0.2], FP32
    shifted, correlators every `every` steps) into the continuous-batching
    server, then the same arrivals through the plain FP64 path (one lattice
    per launch, first come first served)."""
    from paper_1204_6734_amd import inputs as I
    reqs = I.serving_requests(nreq, rate=rate, seed=4)

    def params(r, precision):
        return F.make_params(r["side"], r["side"], precision=precision, ux0=r["ux0"], kT=r["kT"],
                             seed=r["seed"], sample_every=every, block_steps=50)

    def summarize(lat, t_first, t_last, work):
        lat = sorted(lat)
        q = lambda f: lat[min(len(lat) - 1, int(f * len(lat)))]
        span = t_last - t_first
        return {"solves_per_s": len(lat) / span, "p50_latency_s": q(0.5), "p99_latency_s": q(0.99),
                "makespan_s": span, "site_updates_per_s": work / span}

    work = sum(r["side"] ** 2 * r["nsteps"] for r in reqs)
    budget = 64 << 30
    S = F.Server(budget, max_slots=64, chunk_steps=chunk, precision=F.FP32_SHIFTED,
                 threaded=True)
    t0 = time.perf_counter()
    for k, r in enumerate(reqs):
        while time.perf_counter() - t0 < r["t"]:
            time.sleep(0.0005)
        S.submit(params(r, F.FP32_SHIFTED), r["nsteps"], tag=k)
    print(f"serving: {nreq} requests submitted", file=sys.stderr, flush=True)
    last = time.perf_counter()
    while S.stats()["completed"] < nreq:
        time.sleep(0.01)
        if time.perf_counter() - last > 10:
            last = time.perf_counter()
            print(f"serving: {S.stats()['completed']}/{nreq} done", file=sys.stderr, flush=True)
    S.drain()
    print("serving: drained", file=sys.stderr, flush=True)
    res = S.poll(nreq + 8)
    st = S.stats()
    S.close()
    assert len(res) == nreq and all(x["status"] == 0 for x in res)
    # the server clock starts at creation (t0 up to a few microseconds)
    lat = [x["t_done"] - x["t_submit"] for x in res]
    out = {"requests": nreq, "rate_per_s": rate, "chunk_steps": chunk, "sample_every": every,
           "served": summarize(lat, min(x["t_submit"] for x in res),
                               max(x["t_done"] for x in res), work),
           "device_busy_fraction": st["busy_s"] / max(st["wall_s"], 1e-9)}
    if baseline:
        lat0 = []
        t0 = time.perf_counter()
        tfirst = None
        for k, r in enumerate(reqs):
            while time.perf_counter() - t0 < r["t"]:
                time.sleep(0.0005)
            if tfirst is None:
                tfirst = time.perf_counter() - t0
            L = F.Lattice(params(r, F.FP64), stream=torch.cuda.current_stream())
            L.step(r["nsteps"])
            L.covariance()
            L.close()
            lat0.append(time.perf_counter() - t0 - r["t"])
            if (k + 1) % 10 == 0:
                print(f"baseline: {k + 1}/{nreq} done", file=sys.stderr, flush=True)
        out["baseline_fp64_one_per_launch"] = summarize(lat0, tfirst, time.perf_counter() - t0,
                                                        work)
    return out


def run_d3q19(F, torch, steps: int, warmup: int, n: int = 256, precision: str = "fp32"):
    """The D3Q19 generalisation: an n^3 lattice, FP32-shifted (or FP64)
    storage, in the local f-norm basis (u0 = (0.1, 0, 0), kT = 1e-4, tau =
    1), no sampling."""
    fp64 = precision == "fp64"
    p = F.make_params3(n, n, n, precision=F.FP64 if fp64 else F.FP32_SHIFTED, ux0=0.1,
                       kT=1e-4, seed=1)
    L = F.Lattice3(p, stream=torch.cuda.current_stream())
    L.step(warmup)
    L.sync()
    L.profile(True)
    L.kernel_time()
    t0 = time.perf_counter()
    L.step(steps)
    L.sync()
    dt = time.perf_counter() - t0
    kms, launches = L.kernel_time()
    sites = n ** 3
    kernel_ms = kms / max(launches, 1)
    bytes_per_site = 304 if fp64 else 152
    achieved = bytes_per_site * sites / (kernel_ms * 1e-3) / 1e9
    # the kernel is bound by its vector arithmetic: flops per site (from its
    # code) against the vector peak without packed instructions; beside it
    # the HBM fraction of its algorithmic bytes per site, and (FP32) its VALU
    # issue (wavefront instructions per site from the SQ_INSTS_VALU counter)
    flops = D3Q19_FP64_FLOPS_PER_SITE if fp64 else D3Q19_FLOPS_PER_SITE
    peak = FP64_VECTOR_PEAK if fp64 else FP32_VECTOR_PEAK
    tflops = flops * sites / (kernel_ms * 1e-3) / 1e12
    out = {"mlups": sites * steps / dt / 1e6, "ms_per_step": dt * 1e3 / steps,
           "kernel_ms": kernel_ms, "sites": sites, "steps": steps,
           "roofline": {"bound": "alu", "achieved": round(tflops, 2),
                        "peak": round(peak / 1e12, 1), "unit": "TFLOP/s",
                        "frac": round(tflops * 1e12 / peak, 4), "flops_per_site": flops,
                        "kernel": "step3_kernel<%s,fnorm>" % ("double,double" if fp64 else
                                                              "float,float")},
           "hbm": {"achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                   "frac": round(achieved / HBM_PEAK_GBS, 4), "bytes_per_site": bytes_per_site}}
    if not fp64:
        wave_instr = D3Q19_VALU_PER_SITE * sites / 64
        out["valu_issue"] = {"wavefront_instructions_per_site": D3Q19_VALU_PER_SITE,
                             "issue_ms_at_4_cycles": round(wave_instr / VALU_ISSUE_PEAK * 1e3,
                                                           4)}
    return out


def run_config2(F) -> dict:
    """The 256 x 256 mixed-relaxation-time statistics workload, FP64 and
    FP32-shifted, u_x0 in {0, 0.1, 0.2}: the three background flows of one
    precision step side by side (one lattice each, on its own stream,
    replaying captured graphs).  Reports the aggregate rate of the sampled
    steps (each with the correlator sums, every tenth with a structure-factor
    sample) and, per run, the statistical resolution reached (largest
    relative standard error of the moment covariances' diagonal)."""
    from paper_1204_6734_amd import analysis as A
    us = (0.0, 0.1, 0.2)
    out = {}
    for prec, code in (("fp64", F.FP64), ("fp32", F.FP32_SHIFTED)):
        rs = A.mixed_tau_statistics_many(F, code, us)
        dt = rs[0]["seconds"]
        out[f"{prec}_sampled"] = {
            "mlups_aggregate": round(len(us) * 256 * 256 * rs[0]["steps"] / dt / 1e6, 1),
            "seconds": round(dt, 3), "lattices_together": len(us)}
        for u, r in zip(us, rs):
            c = r["cov"]
            d = np.diag(c["cov_m_fnorm_u0"])[3:]
            se = np.diag(c["se_cov_m"])[3:]
            out[f"{prec}_u{u:g}"] = {"nsamples": c["nsamples"], "nblocks": c["nblocks"],
                                     "max_rel_se_diag": float((se / d).max())}
        print(f"config2 {prec}: {out[f'{prec}_sampled']}", file=sys.stderr, flush=True)
    return out


def copy_calibration(reps: int = 5):
    """A plain copy kernel of known size: each launch reads and writes
    exactly 1 GiB.  Its FETCH_SIZE / WRITE_SIZE readings scale the step
    kernel's counters to bytes."""
    import torch
    n = 1 << 28
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "reps": reps}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="large",
                    choices=["large", "ensemble", "serve", "paper", "d3q19", "config2",
                             "cpu"])
    ap.add_argument("--requests", type=int, default=None,
                    help="serving window (default 40 in the main line, 400 with --workload serve)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--nx", type=int, default=8192)
    ap.add_argument("--sk-every", type=int, default=100,
                    help="structure-factor and mode-log interval of the large workload (0: off)")
    ap.add_argument("--rate", type=float, default=50.0, help="serving arrival rate (1/s)")
    ap.add_argument("--launch", default=None,
                    help="TILES,GRID: fix the step launch shape instead of autotuning "
                         "(profiling runs)")
    ap.add_argument("--basis", default="fnorm", choices=sorted(BASES),
                    help="collision basis of the large workload (default: the local f-norm)")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"],
                    help="storage precision of the large workload (default: FP32-shifted)")
    ap.add_argument("--ux0", type=float, default=0.1,
                    help="background velocity of the large workload (above 0.25 the FP32-storage "
                         "collision runs in FP64)")
    ap.add_argument("--sample-every", type=int, default=0,
                    help="correlator sampling interval of the large workload (0: off)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the library steps a "
                                   "lattice on one GPU (its multi-GPU decomposition is a design, "
                                   "not implemented)",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import paper_1204_6734_amd as F
    F.load()
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    if args.workload == "ensemble":
        r = run_ensemble(F, torch, args.steps, args.warmup)
        print(json.dumps({"workload": "64 x 128^2 FP32 ensemble, hipGraph", **r}), flush=True)
        return
    if args.workload == "d3q19":
        r = run_d3q19(F, torch, args.steps, args.warmup, precision=args.precision)
        store = "FP64" if args.precision == "fp64" else "FP32-shifted"
        print(json.dumps({"workload": f"256^3 D3Q19 {store}, f-norm, u_x0=0.1, kT=1e-4, tau=1",
                          **r}), flush=True)
        return
    if args.workload == "paper":
        from paper_1204_6734_amd import analysis as A
        t0 = time.perf_counter()
        r = A.paper_experiments(F)
        print(json.dumps({"workload": "the paper's 21x21 sweeps (Hermite, f-norm local, f-norm "
                                      "table), mu/rho0 = 1e-6", "seconds": time.perf_counter() - t0,
                          **r}), flush=True)
        return
    if args.workload == "cpu":
        print(json.dumps({"workload": "oracle timings of the statistics workloads",
                          **cpu_plan()}), flush=True)
        return
    if args.workload == "config2":
        r = run_config2(F)
        print(json.dumps({"workload": "256x256 D2Q9, u_x0 in {0, 0.1, 0.2}, kT=1e-4, six "
                                      "tau from U[0.6, 1.5], 2e4 + 1e5 steps, correlators "
                                      "every step, S(k) every 10 steps, FP64 and "
                                      "FP32-shifted", **r}), flush=True)
        return
    if args.workload == "serve":
        r = run_serving(F, torch, nreq=args.requests or 400, rate=args.rate)
        print(json.dumps({"workload": f"serving, Poisson {args.rate:g}/s", **r}), flush=True)
        return
    launch = tuple(int(v) for v in args.launch.split(",")) if args.launch else None
    r = run_large(F, torch, args.steps, args.warmup, nx=args.nx, every=args.sk_every,
                  launch=launch, basis=args.basis, precision=args.precision, ux0=args.ux0,
                  sample_every=args.sample_every)
    mlups = r["sites"] * args.steps / r["dt"] / 1e6
    bps = BYTES_PER_SITE[r["dtype"]]
    achieved = bps * r["sites"] / (r["kernel_ms"] * 1e-3) / 1e9
    traffic = traffic_from_profiles(r["kernel_name"])
    # the step's memory traffic with no arithmetic (same layout, tiles and
    # addressing): the practical ceiling of its access pattern; and a plain
    # contiguous copy of the population bytes: the device's streaming ceiling
    copy_ms = r["probes"]["copy_ms"]
    copy_gbps = bps * r["sites"] / (copy_ms * 1e-3) / 1e9
    stream_bytes, stream_ms = r["probes"]["stream_bytes"], r["probes"]["stream_ms"]
    stream_gbps = 2 * stream_bytes / (stream_ms * 1e-3) / 1e9
    out = {
        "metric": "fluct. D2Q9 MLUPS, % of HBM roofline; served solves/s + p99 latency",
        "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(r["dt"] * 1e3 / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": r["dtype"],
        "data": "synthetic", "config": r["config"],
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": r["kernel_label"],
                     "bytes_per_site": bps, "kernel_ms": round(r["kernel_ms"], 4),
                     "launches": r["launches"],
                     "copy_probe": {"GBps": round(copy_gbps, 1), "ms": round(copy_ms, 4),
                                    "frac_of_peak": round(copy_gbps / HBM_PEAK_GBS, 4),
                                    "kernel_frac_of_copy": round(achieved / copy_gbps, 4),
                                    "what": "the step's loads and stores, no arithmetic"},
                     "stream_copy": {"GBps": round(stream_gbps, 1), "ms": round(stream_ms, 4),
                                     "frac_of_peak": round(stream_gbps / HBM_PEAK_GBS, 4),
                                     "what": "contiguous copy of the population bytes, "
                                             "16 B per thread"}},
        "pct_hbm_roofline": round(100 * mlups * 1e6 * bps / (HBM_PEAK_GBS * 1e9), 2),
        "launch": dict(r["launch"], settle_steps=r["settle_steps"]),
        "structure_factor": {"sk_every": args.sk_every, "sk_samples_in_window": r["sk_in_window"],
                             "mode_logs_in_window": r["mode_logs_in_window"],
                             "with_sk": r["with_sk"]},
    }
    if not args.no_serving:
        out["serving"] = run_serving(F, torch, nreq=args.requests or 40)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds, BASES[args.basis][1], args.ux0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
