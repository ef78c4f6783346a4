"""Benchmark of the particle step on one MI355X.

Workload (default): relativistic pair plasma, 256^3 periodic cells, 32 particles per cell per
species (1,073,741,824 particles), Maxwell-Juettner momenta at kT = m c^2, cubic weights,
6th-order fields, dt = 0.4, generated in device memory.  A step is one pass of the whole
particle step: gather/push/deposit (+ high-order line solve), sort by cell, field step.

Prints one JSON line: value = particle updates/s of the split-precision FP32 path over the
timed steps (inputs resident in HBM before timing starts); the FP64 plain form is timed on
the same workload for comparison; ``roofline`` describes the dominant kernel (the tiled
gather/push/deposit kernel) with its launch time measured by HIP events on its own stream;
``cpu_baseline`` times the FP64 CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

SEED = 12114575
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_pair_mj_run(pp, ind, torch, n, ppc, theta, split, with_id=False, rad_tau=0.0, current_scheme=0,
                     gauss_passes=0, time_order=2):
    """Build a pp.Run for the pair-plasma workload with particles generated on the device.
    Returns the run and the number of particles per species."""
    npart = n[0] * n[1] * n[2] * ppc
    dev = torch.device("cuda:0")
    rt = torch.float32 if split else torch.float64
    cells = [torch.empty(npart, dtype=torch.int32, device=dev) for _ in range(2)] if split else None
    offs = [torch.empty((3, npart), dtype=rt, device=dev) for _ in range(2)]
    us = [torch.empty((3, npart), dtype=rt, device=dev) for _ in range(2)]
    st = torch.cuda.current_stream().cuda_stream
    chunk = 1 << 26
    for start in range(0, npart, chunk):
        cnt = min(chunk, npart - start)
        ind.pair_maxwell_juttner(SEED, n, start, cnt, theta, ind.split_mode(split, 3),
                                 [c[start:] for c in cells] if split else None,
                                 [[o[d, start:] for d in range(3)] for o in offs],
                                 [[u[d, start:] for d in range(3)] for u in us], st)
    torch.cuda.synchronize()
    params = pp.make_params(n, shape_order=3, field_order=6, dt=0.4, alpha=0.55,
                            precision=pp.PP_PREC_FP32_SPLIT if split else pp.PP_PREC_FP64,
                            relax_tol=1e-8 if split else 1e-14, relax_max_iter=100, rad_tau=rad_tau,
                            current_scheme=current_scheme, gauss_filter_passes=gauss_passes, time_order=time_order)
    species = []
    for s, q in enumerate((-1.0, 1.0)):
        sp = dict(q=q, m=1.0, w=1.0 / ppc, u=us[s])
        if split:
            sp.update(cell=cells[s], off=offs[s])
        else:
            sp.update(pos=offs[s])
        species.append(sp)
    run = pp.Run(params, species, with_id=with_id)
    del cells, offs, us
    return run, npart


def time_steps(run, torch, steps, warmup):
    for _ in range(warmup):
        run.step()
    torch.cuda.synchronize()
    run.timing(True)
    t0 = time.perf_counter()
    for i in range(steps):
        run.step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_gpd, launches = run.timing_read()
    run.timing(False)
    return (t1 - t0), ms_gpd / max(launches, 1)


def host_cpu():
    """CPU model (from /proc/cpuinfo) and the number of cores this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0))


def time_oracle(wl, steps, openmp, progress=None):
    """Seconds for `steps` whole oracle steps of workload `wl` (plain scalar build, or the
    OpenMP build with one current buffer per thread) and the threads used.  With `progress`,
    the step is taken species by species as the oracle's own step does (particles of every
    species, high-order current, field step; leapfrog order only) and progress(text) is
    called after each species."""
    from oracle import orc
    orc.build()
    P = orc.make_params(**wl.params())
    run = orc.Run(P, [dict(q=s.q, m=s.m, w=s.w, pos=s.pos, u=s.u) for s in wl.species])

    def one_step(k):
        if progress is None or P.time_order == 4:
            run.step()
            return
        run.J[:] = 0.0
        for i, s in enumerate(run.species):
            run.flags |= orc.step_species_kd(P, P.dt, s["q"], s["m"], s["w"], s["pos"], s["u"], run.E, run.B, run.J)
            progress(f"step {k + 1}/{steps}, species {i + 1}/{len(run.species)}")
        if P.current_scheme == 0:
            orc.current_high_order(P, run.J)
        run.fields_step()
        run.nstep += 1

    if openmp:
        with orc.openmp():
            threads = orc.num_threads()
            t0 = time.perf_counter()
            for k in range(steps):
                one_step(k)
            dt = time.perf_counter() - t0
    else:
        threads = 1
        t0 = time.perf_counter()
        for k in range(steps):
            one_step(k)
        dt = time.perf_counter() - t0
    return dt, threads


def cpu_baseline(n_sample=(24, 24, 24), ppc=32, steps_one=1, steps_all=3):
    """The FP64 CPU oracle, as it stands, on the host cores of this machine, on a bounded
    sample of the benchmark's workload (pair plasma, Maxwell-Juettner kT = mc^2, cubic weights,
    6th-order fields, same particles per cell) in a smaller box: the plain scalar build on one
    core and the OpenMP build (one current buffer per thread) on every core this process may
    use.  `value` is the all-core rate; the one-core rate is reported beside it."""
    from paper_1211_4575_amd import inputs as I
    model, cores = host_cpu()
    os.environ.setdefault("OMP_NUM_THREADS", str(cores))
    wl = I.pair_maxwell_juttner(n=n_sample, ppc=ppc, theta=1.0)
    t1, _ = time_oracle(wl, steps_one, openmp=False)
    tn, threads = time_oracle(wl, steps_all, openmp=True)
    one = wl.n_particles * steps_one / t1
    allc = wl.n_particles * steps_all / tn
    return dict(value=allc, unit="particle updates/s", cores=threads, kind="oracle",
                sample=f"{n_sample[0]}x{n_sample[1]}x{n_sample[2]} box of the same workload ({wl.n_particles} particles): "
                       f"{steps_all} whole steps on {threads} threads (OpenMP build, {tn:.1f} s) and {steps_one} on one "
                       f"core (plain build, {t1:.1f} s)",
                one_core=one, cpu_model=model, nproc=cores)


def cpu_plan():
    """The whole CPU-baseline plan (a long run, not part of the default benchmark): the plain
    heating workload in full (16^3, 8 per cell per species, TSC, 2nd-order fields, 100 steps),
    the two-stream workload (128x32x32, cubic, 6th order) and the pair plasma at 64^3 (32 per
    cell per species, cubic, 6th order) for 20 steps, each on one core (plain build) and on
    every core (OpenMP build)."""
    from paper_1211_4575_amd import inputs as I
    model, cores = host_cpu()
    os.environ.setdefault("OMP_NUM_THREADS", str(cores))
    out = {"cpu_model": model, "nproc": cores, "runs": []}
    plans = [("plain heating 16^3, TSC, 2nd order, 100 steps", I.plain_heating(), 100, 100),
             ("two-stream 128x32x32, 32 ppc per beam, cubic, 6th order, 20 steps (one core: 1 step)",
              I.two_stream(), 1, 20),
             ("pair plasma 64^3, 32 ppc/species, cubic, 6th order, 20 steps (one core: 1 step)",
              I.pair_maxwell_juttner(n=(64, 64, 64), ppc=32, theta=1.0), 1, 20)]
    for name, wl, s1, sn in plans:
        def progress(text, name=name):
            log(f"[cpu-plan] {name}: {text}")
        t1, _ = time_oracle(wl, s1, openmp=False, progress=progress)
        log(f"[cpu-plan] {name}: one core {wl.n_particles * s1 / t1:.3e} updates/s ({t1:.1f} s)")
        tn, threads = time_oracle(wl, sn, openmp=True, progress=progress)
        log(f"[cpu-plan] {name}: {threads} threads {wl.n_particles * sn / tn:.3e} updates/s ({tn:.1f} s)")
        out["runs"].append(dict(workload=name, particles=wl.n_particles, one_core=dict(steps=s1, s=t1,
                                updates_per_s=wl.n_particles * s1 / t1),
                                all_cores=dict(threads=threads, steps=sn, s=tn, updates_per_s=wl.n_particles * sn / tn)))
    print(json.dumps(out), flush=True)
    return 0


def flops_per_update(O=3, direct=False):
    """Algorithmic floating-point operations of one particle update (FMA = 2), counted from the
    method as the tiled kernel formulates it: B-spline weight sets (centred and staggered at
    the old position, centred at the new one; 3 axes; ~17 flops each for cubic), factored
    gather of 6 components, Vay push, move, and per current component the weight changes,
    prefix sum, the two factors of F, F itself and the (O+1)(O+2)^2 products."""
    n1, n2 = O + 1, O + 2
    weights = 9 * (17 if O == 3 else 9)
    gather = 6 * 2 * (n1 ** 3 + n1 ** 2 + n1)
    push = 100
    move = 12
    if direct:  # centred and staggered weight sets at the time-centred position, 2 flops per product
        return weights - 3 * (17 if O == 3 else 9) + 6 * (17 if O == 3 else 9) + gather + push + move + \
            3 * (2 * n1 * n1 * n1 + 2 * n1 * n1 + 1)
    per_comp = n2 + (n1 - 1) + 2 * n2 + 3 * n2 + 3 * n2 * n2 + 2 * n1 * n2 * n2
    return weights + gather + push + move + 3 * per_comp


# LDS rate measured on gfx950 by bench_lds_rates.hip (python bench.py --lds-probe): 6.3 clk
# per CU for one 64-lane 64-bit integer atomic add with aligned, distinct addresses.
LDS_CLK_PER_WAVE_ATOMIC = 6.3
CUS, CLOCK_HZ = 256, 2.4e9


BYTES_PER_UPDATE = 56.0  # split state read + written: int32 cell + 3 FP32 offsets + 3 FP32 u


def kernel_roofline(npart, gpd_ms, direct=False):
    """The dominant kernel against three ceilings.  Primary: HBM, algorithmic bytes (56 per
    particle update) over the live launch time against 8 TB/s, with the counted traffic when
    the committed counter summary matches these kernel sources.  From the same summary: VALU,
    counted wavefront instructions over the launch time against one per clock per CU (the
    unpacked rate: the build turns packed FP32 off, and FP64 FMA issues at that rate too), and
    LDS atomics, counted ds_add instructions over the launch time against the rate the LDS
    probe measures for aligned 64-lane 64-bit adds."""
    sec = gpd_ms * 1e-3
    achieved_gbs = npart * BYTES_PER_UPDATE / sec / 1e9
    traffic = measured_traffic(npart)
    cs = read_counter_summary(npart)
    out = {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved_gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": "k_gpd32<3>",
           "gpd_ms": round(gpd_ms, 3), "algorithmic_bytes_per_launch": npart * BYTES_PER_UPDATE,
           "flop_per_update_model": flops_per_update(3, direct=direct)}
    if cs is not None and (cs.get("copy_gbs") or cs.get("ew_gbs")):
        # against the best rate a plain stream kernel (4 GiB read + written: the device copy, and
        # an elementwise pass) reached in the counter runs
        best = max(cs.get("copy_gbs", 0.0), cs.get("ew_gbs", 0.0))
        out["stream_peak_gbs"] = round(best, 1)
        out["frac_of_stream"] = round(achieved_gbs / best, 4)
    if cs is None or "valu_insts_per_launch" not in cs:
        out["valu"] = out["lds_atomic"] = None
        out["counters"] = "no counter summary for these kernel sources"
        return out
    valu_peak = CUS * CLOCK_HZ  # wavefront instructions/s, one per clock per CU
    v = cs["valu_insts_per_launch"] / sec
    out["valu"] = {"bound": "alu", "achieved": v, "peak": valu_peak, "unit": "VALU wavefront instr/s",
                   "frac": round(v / valu_peak, 4), "insts_per_64_particles": round(cs["valu_insts_per_launch"] * 64 / npart, 1)}
    if "lds_atomic_insts_per_launch" in cs:
        lds_peak = CUS * CLOCK_HZ / LDS_CLK_PER_WAVE_ATOMIC
        la = cs["lds_atomic_insts_per_launch"] / sec
        out["lds_atomic"] = {"bound": "lds", "achieved": la, "peak": lds_peak, "unit": "ds_add wavefront instr/s",
                             "frac": round(la / lds_peak, 4),
                             "atomics_per_64_particles": round(cs["lds_atomic_insts_per_launch"] * 64 / npart, 1),
                             "lds_insts_per_64_particles": round(cs.get("lds_insts_per_launch", float("nan")) * 64 / npart, 1)}
    if "lds_active_per_launch" in cs and "gui_active_per_launch" in cs:
        # fraction of the kernel's CU cycles in which the LDS pipe was busy (all LDS instructions,
        # bank conflicts included), from the same counter runs
        busy = cs["lds_active_per_launch"] / (cs["gui_active_per_launch"] / XCDS * CUS)
        if out.get("lds_atomic"):
            out["lds_atomic"]["lds_pipe_busy"] = round(busy, 4)
    fr = {"hbm": out["frac"], "valu": out["valu"]["frac"],
          "lds": (out.get("lds_atomic") or {}).get("lds_pipe_busy", (out.get("lds_atomic") or {}).get("frac", 0.0))}
    out["binding"] = max(fr, key=fr.get)
    out["counters"] = f"profiles/k_gpd32_pair_mj_256_counters.md, digest {cs.get('kernel_source_digest', '')}"
    return out


def kernel_source_digest():
    """Digest of the sources of the dominant kernel (so stored counter figures are only used
    while the kernel they were taken on is unchanged)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("pp_gpd32.hip", "pp_device.hpp", "pp_internal.hpp"):
        h.update(open(os.path.join(ROOT, "paper_1211_4575_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(particles):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE, each divided by what the same counter reads per byte of a plain
    copy of known size), or None when the summary is missing, for another workload, or was
    taken on other kernel sources."""
    v = read_counter_summary(particles)
    try:
        f = v["fetch_kib_per_launch"] * 1024.0 / (v["copy_fetch_kib"] * 1024.0 / v["copy_bytes"])
        w = v["write_kib_per_launch"] * 1024.0 / (v["copy_write_kib"] * 1024.0 / v["copy_bytes"])
        return f + w
    except (TypeError, KeyError, ZeroDivisionError):
        return None


def read_counter_summary(particles):
    """Figures of the committed rocprofv3 counter summary of the dominant kernel (per launch), or
    None when the summary is missing, for another workload, or was taken on other kernel
    sources."""
    path = os.path.join(ROOT, "profiles", "k_gpd32_pair_mj_256_counters.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        line = line.strip()
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            vals[k.strip()] = v.strip()
    try:
        if vals.get("kernel_source_digest") != kernel_source_digest() or int(vals["particles"]) != particles:
            return None
        out = {k: float(v) for k, v in vals.items() if k != "kernel_source_digest"}
        out["kernel_source_digest"] = vals["kernel_source_digest"]
        return out
    except (KeyError, ValueError):
        return None


def _pmc_rows(d):
    """(kernel name, dispatch id) -> {counter: value summed over the rows of that dispatch},
    and the same key -> kernel duration in ms, from one rocprofv3 --pmc output folder."""
    import csv
    import glob
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    agg, dur = {}, {}
    for f in files:
        for r in csv.DictReader(open(f)):
            key = (r["Kernel_Name"], int(r["Dispatch_Id"]))
            c = agg.setdefault(key, {})
            c[r["Counter_Name"]] = c.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
            dur[key] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6
    return agg, dur


XCDS = 8  # GRBM_GUI_ACTIVE comes summed over the accelerator's XCDs


def counter_summary(dirs, out, particles, cmds):
    """Write the counter summary of the dominant kernel (the cubic 4x4x4-tile particle kernel,
    launches after the first, which follows the initial sort) from rocprofv3 --pmc folders:
    HBM bytes (FETCH_SIZE, WRITE_SIZE, calibrated on the largest device copy of the same runs)
    and the instruction and LDS counters, per launch, with the digest of the kernel's sources."""
    import statistics
    per, copy, ew, times = {}, {}, {}, []
    for d in dirs:
        agg, dur = _pmc_rows(d)
        launches = sorted((k for k in agg if "k_gpd32<3, pp::TileCT<3, 4, 4, 4, false>" in k[0]), key=lambda k: k[1])
        for key in launches[1:]:
            for cname, v in agg[key].items():
                per.setdefault(cname, []).append(v)
            times.append(dur[key])
        # the calibration copy (4 GiB, about 2 ms) is by far the longest device copy of its runs;
        # the passes without one only have copies of a few kilobytes
        copies = [k for k in agg if "copyBuffer" in k[0]]
        if copies:
            big = max(copies, key=lambda k: dur[k])
            if dur[big] > 0.5:
                copy.update(agg[big])
                copy["copy_ms"] = max(copy.get("copy_ms", 0.0), dur[big])
        # the elementwise pass over the same 4 GiB (torch's negation kernel, which splits a
        # tensor this large into several dispatches: their counters and times are summed)
        ews = [k for k in agg if "neg_kernel" in k[0] and dur[k] > 0.1]
        if ews:
            tot = {}
            for k in ews:
                for cname, v in agg[k].items():
                    tot[cname] = tot.get(cname, 0.0) + v
            ew.update(tot)
            ew["ms"] = max(ew.get("ms", 0.0), sum(dur[k] for k in ews))
            ew["dispatches"] = len(ews)
    mean = {k: statistics.fmean(v) for k, v in per.items()}
    ms = statistics.median(times)
    n64 = particles / 64.0
    lines = ["# k_gpd32 — counters of the particle kernel, pair plasma 256^3, 32 ppc/species", "",
             "Commands (one rocprofv3 pass each; every pass runs the benchmark for one warm-up and one timed step,"
             " and the figures are means over the kernel's launches after the first):", "", "```"]
    lines += list(cmds) + ["```", ""]
    if "SQ_INSTS_VALU" in mean:
        lines.append(f"Per 64 particles (one wavefront's share): {mean['SQ_INSTS_VALU'] / n64:.0f} VALU instructions; "
                     f"{mean.get('SQ_INSTS_LDS', float('nan')) / n64:.0f} LDS instructions, of which "
                     f"{mean.get('SQ_INSTS_LDS_ATOMIC', float('nan')) / n64:.0f} atomics.")
    if "GRBM_GUI_ACTIVE" in mean:
        cyc = mean["GRBM_GUI_ACTIVE"] / XCDS * CUS
        parts = [f"{label} {100 * mean[c] / cyc:.0f} %" for c, label in
                 (("SQ_INSTS_VALU", "VALU issue (instructions / CU cycles)"), ("SQ_ACTIVE_INST_VALU", "VALU active"),
                  ("SQ_LDS_IDX_ACTIVE", "LDS active"), ("SQ_LDS_BANK_CONFLICT", "LDS bank-conflict cycles"),
                  ("SQ_ACTIVE_INST_LDS", "LDS instruction active"), ("SQ_BUSY_CU_CYCLES", "CU busy"))
                 if c in mean]
        lines.append(f"CU cycles per launch: GRBM_GUI_ACTIVE / {XCDS} XCDs x {CUS} CUs = {cyc:.4g}; per CU cycle: "
                     + ", ".join(parts) + ".")
    if "FETCH_SIZE" in mean and "FETCH_SIZE" in copy:
        cb = 4 * (1 << 30)
        fb = mean["FETCH_SIZE"] / (copy["FETCH_SIZE"] / cb)
        line = f"HBM traffic per launch: FETCH {fb / 1e9:.2f} GB"
        if "WRITE_SIZE" in mean and "WRITE_SIZE" in copy:
            wb = mean["WRITE_SIZE"] / (copy["WRITE_SIZE"] / cb)
            line += f", WRITE {wb / 1e9:.2f} GB, total {(fb + wb) / 1e9:.2f} GB"
        line += (f", against {BYTES_PER_UPDATE * particles / 1e9:.2f} GB algorithmic (56 B per particle update). "
                 f"Calibration: the 4 GiB device copy (`__amd_rocclr_copyBuffer`, reads and writes 4 GiB) reads "
                 f"FETCH_SIZE {copy['FETCH_SIZE']:.6g} KiB and WRITE_SIZE {copy.get('WRITE_SIZE', float('nan')):.6g} KiB; "
                 f"a kernel's counter is divided by the copy's counter per byte.")
        lines.append(line)
    if "FETCH_SIZE" in ew or "WRITE_SIZE" in ew:
        cb = 4 * (1 << 30)
        parts = []
        if "FETCH_SIZE" in ew:
            parts.append(f"FETCH_SIZE {ew['FETCH_SIZE']:.6g} KiB (factor {ew['FETCH_SIZE'] * 1024 / cb:.3f})")
        if "WRITE_SIZE" in ew:
            parts.append(f"WRITE_SIZE {ew['WRITE_SIZE']:.6g} KiB (factor {ew['WRITE_SIZE'] * 1024 / cb:.3f})")
        line = (f"Second calibration: an elementwise pass over the same 4 GiB (torch's negation kernel: plain "
                f"vector loads and stores, {int(ew.get('dispatches', 1))} dispatches) reads " + " and ".join(parts))
        if "FETCH_SIZE" in mean and "FETCH_SIZE" in ew:
            f2 = mean["FETCH_SIZE"] / (ew["FETCH_SIZE"] / cb)
            line += f"; against it the particle kernel fetches {f2 / 1e9:.2f} GB per launch"
        if "ms" in ew:
            line += (f". It streams its 8 GiB in {ew['ms']:.3f} ms, {2 * cb / (ew['ms'] * 1e-3) / 1e12:.2f} TB/s"
                     + (f", against {2 * cb / (copy['copy_ms'] * 1e-3) / 1e12:.2f} TB/s for the device copy"
                        if "copy_ms" in copy else ""))
        lines.append(line + ".")
    lines += ["", f"Kernel time under the profiler (median of those launches): {ms:.3f} ms.", "",
              "Machine-read by bench.py (used only while the kernel sources are unchanged):", "",
              f"- kernel_source_digest: {kernel_source_digest()}", f"- particles: {particles}", f"- kernel_ms: {ms:.6g}"]
    keymap = {"FETCH_SIZE": "fetch_kib_per_launch", "WRITE_SIZE": "write_kib_per_launch",
              "SQ_INSTS_VALU": "valu_insts_per_launch", "SQ_INSTS_LDS": "lds_insts_per_launch",
              "SQ_INSTS_LDS_ATOMIC": "lds_atomic_insts_per_launch", "SQ_ACTIVE_INST_VALU": "valu_active_per_launch",
              "SQ_ACTIVE_INST_LDS": "lds_inst_active_per_launch", "SQ_LDS_IDX_ACTIVE": "lds_active_per_launch",
              "SQ_LDS_BANK_CONFLICT": "lds_conflict_per_launch", "SQ_WAVE_CYCLES": "wave_cycles_per_launch",
              "SQ_BUSY_CYCLES": "sq_busy_cycles_per_launch", "SQ_BUSY_CU_CYCLES": "cu_busy_cycles_per_launch",
              "GRBM_GUI_ACTIVE": "gui_active_per_launch"}
    for cname, key in keymap.items():
        if cname in mean:
            lines.append(f"- {key}: {mean[cname]:.6g}")
    if "FETCH_SIZE" in copy:
        lines += [f"- copy_bytes: {4 * (1 << 30)}", f"- copy_fetch_kib: {copy['FETCH_SIZE']:.6g}"]
        if "WRITE_SIZE" in copy:
            lines.append(f"- copy_write_kib: {copy['WRITE_SIZE']:.6g}")
    if "copy_ms" in copy:
        # the device copy reads and writes its bytes: the HBM rate a plain stream reaches here
        lines.append(f"- copy_gbs: {2 * 4 * (1 << 30) / (copy['copy_ms'] * 1e-3) / 1e9:.6g}")
    if "FETCH_SIZE" in ew:
        lines.append(f"- ew_fetch_kib: {ew['FETCH_SIZE']:.6g}")
    if "WRITE_SIZE" in ew:
        lines.append(f"- ew_write_kib: {ew['WRITE_SIZE']:.6g}")
    if "ms" in ew:
        lines.append(f"- ew_gbs: {2 * 4 * (1 << 30) / (ew['ms'] * 1e-3) / 1e9:.6g}")
    open(out, "w").write("\n".join(lines) + "\n")
    return out


def stats_summary(d, out, particles, cmd):
    """Write the kernel-time summary of one rocprofv3 --kernel-trace --stats folder: the stats
    table, then the median duration of each kernel over the calls of the steady-state steps
    (every call after the particle kernel's first launch)."""
    import csv
    import glob
    import statistics
    st = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)
    tr = glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)
    if not st or not tr:
        raise FileNotFoundError(f"no kernel_stats.csv / kernel_trace.csv under {d}")
    lines = [f"# k_gpd32 and the step kernels — kernel times, pair plasma 256^3, 32 ppc/species ({particles:,} particles)",
             "", "Command (on one MI355X; the benchmark's own step count):", "", "```", cmd, "```", "",
             "rocprofv3 `--stats` summary (all calls: includes the one-time generation and first sort from random "
             "order, the first push after it, and the diagnostics after the timed steps):", "",
             "| Kernel | Calls | Average ms | Min ms | Max ms | % |", "|---|---|---|---|---|---|"]
    for r in csv.DictReader(open(st[0])):
        if float(r["Percentage"]) < 0.05:
            continue
        lines.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']) * 1e-6:.3f} | "
                     f"{float(r['MinNs']) * 1e-6:.3f} | {float(r['MaxNs']) * 1e-6:.3f} | {float(r['Percentage']):.2f} |")
    calls = sorted(csv.DictReader(open(tr[0])), key=lambda r: int(r["Start_Timestamp"]))
    gpd = [i for i, r in enumerate(calls) if "k_gpd32<3, pp::TileCT<3, 4, 4, 4, false>" in r["Kernel_Name"]]
    per = {}
    for r in calls[gpd[0] + 1:] if gpd else []:
        per.setdefault(r["Kernel_Name"], []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6)
    lines += ["", "Steady state: median duration per kernel over the calls after the particle kernel's first launch "
              "(that launch follows the initial sort from random order):", "", "| Kernel | median ms | calls |",
              "|---|---|---|"]
    for name, v in per.items():
        lines.append(f"| `{name[:90]}` | {statistics.median(v):.3f} | {len(v)} |")
    if gpd:
        g = [(int(calls[i]["End_Timestamp"]) - int(calls[i]["Start_Timestamp"])) * 1e-6 for i in gpd]
        lines += ["", f"k_gpd32<3> over its {len(g)} launches: first {g[0]:.3f} ms, then median "
                      f"{statistics.median(g[1:]):.3f} ms.  bench.py times the same kernel live with HIP events on "
                      f"its launch stream over the timed steps."]
    open(out, "w").write("\n".join(lines) + "\n")
    return out


def two_stream_rate(k, v0, wb2=0.5):
    """Growth rate at wavenumber k of the symmetric cold relativistic two-stream instability
    (two beams at +-v0, each of plasma frequency^2 wb2, longitudinal mass gamma0^3 m): the
    unstable root of 1 = wb2/gamma0^3 [1/(w - k v0)^2 + 1/(w + k v0)^2], i.e. with
    a = wb2/gamma0^3 and x = k v0, gamma^2 = sqrt(a^2 + 4 a x^2) - x^2 - a."""
    a = wb2 * (1.0 - v0 * v0) ** 1.5
    x2 = (k * v0) ** 2
    g2 = math.sqrt(a * a + 4.0 * a * x2) - x2 - a
    return math.sqrt(g2) if g2 > 0 else 0.0


def growth_rate_fit(t, w, width=4.0):
    """Growth rate of the field amplitude (half the log slope of the E_x energy W) in the linear
    phase, which starts when W first exceeds 10x its mean over t <= 2 and ends when W first
    reaches 10 % of its maximum.  Returns (largest least-squares rate over windows of the given
    width inside that phase, least-squares rate over the whole phase, phase (t0, t1))."""
    import numpy as np
    t = np.asarray(t, dtype=float)
    w = np.asarray(w, dtype=float)
    base = w[t <= 2.0].mean()
    i0 = int(np.argmax(w > 10.0 * base))
    i1 = int(np.argmax(w >= 0.1 * w.max()))
    nan = float("nan")
    if not (w[i0] > 10.0 * base) or i1 <= i0 + 2:
        return nan, nan, (float(t[i0]), float(t[i1]))
    lw = np.log(np.maximum(w, np.finfo(float).tiny))
    whole = 0.5 * float(np.polyfit(t[i0:i1 + 1], lw[i0:i1 + 1], 1)[0])
    best = nan
    j = i0
    while j < i1:
        k = int(np.searchsorted(t, t[j] + width))
        if k > i1 + 1:
            break
        if k - j >= 3:
            r = 0.5 * float(np.polyfit(t[j:k], lw[j:k], 1)[0])
            best = r if not (best >= r) else best
        j += max(1, (k - j) // 8)
    return best, whole, (float(t[i0]), float(t[i1]))


def run_two_stream(torch, pp, ind, n, per_dim, v_beam, uth, steps, split, dx=0.1, cfl=0.4, seed=SEED):
    """Two-stream run generated on the device; returns (times, E_x energy per step, wall s,
    particles)."""
    npart = n[0] * n[1] * n[2] * per_dim[0] * per_dim[1] * per_dim[2]
    dev = torch.device("cuda:0")
    rt = torch.float32 if split else torch.float64
    cells = [torch.empty(npart, dtype=torch.int32, device=dev) for _ in range(2)] if split else None
    offs = [torch.empty((3, npart), dtype=rt, device=dev) for _ in range(2)]
    us = [torch.empty((3, npart), dtype=rt, device=dev) for _ in range(2)]
    ind.two_stream_lattice(seed, 2, n, per_dim, v_beam, uth, ind.split_mode(split, 3), cells,
                           [[o[d] for d in range(3)] for o in offs], [[u[d] for d in range(3)] for u in us],
                           torch.cuda.current_stream().cuda_stream)
    ppc = per_dim[0] * per_dim[1] * per_dim[2]
    species = []
    for s in range(2):
        sp = dict(q=-1.0, m=1.0, w=0.5 / ppc, u=us[s])
        sp.update(dict(cell=cells[s], off=offs[s]) if split else dict(pos=offs[s]))
        species.append(sp)
    P = pp.make_params(n, d=(dx, dx, dx), dt=cfl * dx, shape_order=3, field_order=6, alpha=0.55,
                       precision=pp.PP_PREC_FP32_SPLIT if split else pp.PP_PREC_FP64,
                       relax_tol=1e-8 if split else 1e-14, relax_max_iter=100, rho_background=1.0)
    run = pp.Run(P, species, with_id=False)
    del cells, offs, us
    t, w = [0.0], [run.diagnostics(pp.PP_DIAG_FIELDS).field_Ex]
    t0 = time.perf_counter()
    for i in range(steps):
        run.step()
        w.append(run.diagnostics(pp.PP_DIAG_FIELDS).field_Ex)
        t.append((i + 1) * cfl * dx)
        if (i + 1) % 500 == 0:
            log(f"[two-stream] {'FP32' if split else 'FP64'} step {i + 1}/{steps}, W_Ex {w[-1]:.3e}")
    wall = time.perf_counter() - t0
    d = run.diagnostics(pp.PP_DIAG_ALL)
    run.close()
    torch.cuda.empty_cache()
    return t, w, wall, 2 * npart, d


def two_stream_bench(args, torch, pp):
    """The cold-beam / two-stream test: 128x32x32 cells of 0.1 c/w_pe, two electron beams at
    +-0.2c (32 particles per cell each, quiet lattice, u_th = 0.01c) over a fixed ion
    background, cubic weights, 6th-order fields, 2000 steps of 0.04; growth rate of the E_x
    energy, FP64 then FP32, against linear theory at the box mode nearest the fastest one."""
    from paper_1211_4575_amd import inputs_device as ind
    n, per_dim, v0 = (args.grid_x, 32, 32), (4, 4, 2), 0.2
    L = n[0] * 0.1
    kmax = math.sqrt(3.0) / 2.0 * math.sqrt(0.5) * (1 - v0 * v0) ** 0.75 / v0
    m = max(1, round(kmax * L / (2 * math.pi)))
    theory = two_stream_rate(2 * math.pi * m / L, v0)
    out = {"metric": "two-stream growth rate of the E_x energy / linear theory", "theory_rate": theory,
           "theory_mode": m, "theory_max": math.sqrt(0.5) * (1 - v0 * v0) ** 0.75 / 2}
    for split in ((False, True) if not args.no_fp64 else (True,)):
        t, w, wall, npart, d = run_two_stream(torch, pp, ind, n, per_dim, v0, 0.01, args.ts_steps, split)
        rate, whole, window = growth_rate_fit(t, w)
        key = "fp32_split" if split else "fp64_plain"
        if args.save_history:
            import numpy as np
            np.savez(f"{args.save_history}_{key}.npz", t=np.asarray(t), w=np.asarray(w))
        out[key] = {"rate": rate, "rate_over_theory": rate / theory, "linear_phase": window,
                    "rate_whole_phase": whole,
                    "updates_per_s": npart * args.ts_steps / wall, "wall_s": wall,
                    "final_gauss_rel": d.gauss_max / d.rho_ref, "flags": d.flags}
        log(f"[two-stream] {key}: {out[key]}")
    print(json.dumps(out), flush=True)
    return 0


# The six schemes of the paper's mixed-mode comparison (its table of orders): field order,
# weight order (TSC = quadratic), charge-conserving current, time order.  The runs without
# charge conservation use the direct current with the Gauss-law filter of the original code,
# five passes per step (the paper runs it 5 to 10 times).
MMI_SCHEMES = {1: (2, 2, False, 2), 2: (2, 3, False, 2), 3: (6, 2, False, 2), 4: (6, 3, False, 2),
               5: (6, 3, True, 2), 6: (6, 3, True, 4)}


def run_mmi(torch, pp, ind, g, ppc, steps, T_b, T_p, box=12.8, cfl=0.4, progress=250, kmax_index=16, scheme=5,
            quiet=False, lattice=None):
    """Mixed-mode two-stream run on g^3 cells of a cubic box of ``box`` skin depths, generated
    on the device (FP32 split form).  Returns (times, energies [steps + 1, 4], wall s,
    particles, final diagnostics, (sample times, wave-number indices, bin energies)): per step
    the energy of E projected on the MMI direction (74 degrees from the beam: |E_perp| sin +
    E_z cos), of E_z (the same projection at 0 degrees, the TSI direction), of the x-y mean
    of E_z (wave vectors along the beam), and the volume integral of the projection itself
    (the paper's formula read literally, linear in E); every half time unit (NaN otherwise) the
    longitudinal field energy E.k/|k| of the Fourier modes 60-80 degrees from the beam with
    1 <= |k| <= 8, and the longitudinal energy of every single Fourier mode whose indices are
    all within kmax_index (the bin energies, for rates mode by mode).  ``quiet``: the loader's
    quiet start (pairs of particles with opposite thermal velocities); ``lattice``: its lattice
    positions (points per cell and axis)."""
    import numpy as np

    from paper_1211_4575_amd import inputs as I
    n, dx = (g, g, g), box / g
    dt = cfl * dx
    npart = n[0] * n[1] * n[2] * ppc
    fo, O, cc, torder = MMI_SCHEMES[scheme]
    dev = torch.device("cuda:0")
    cells = [torch.empty(npart, dtype=torch.int32, device=dev) for _ in range(4)]
    offs = [torch.empty((3, npart), dtype=torch.float32, device=dev) for _ in range(4)]
    us = [torch.empty((3, npart), dtype=torch.float32, device=dev) for _ in range(4)]
    st = torch.cuda.current_stream().cuda_stream
    chunk = 1 << 25
    for start in range(0, npart, chunk):
        cnt = min(chunk, npart - start)
        ind.mmi(SEED, n, start, cnt, 4.0, T_b, T_p, 1836.0, ind.split_mode(True, O), [c[start:] for c in cells],
                [[o[d, start:] for d in range(3)] for o in offs], [[u[d, start:] for d in range(3)] for u in us], st,
                quiet=quiet, lattice=lattice)
    species = []
    for s, (nm, q, ion, beam) in enumerate(I.MMI_SPECIES):
        species.append(dict(q=q, m=1836.0 if ion else 1.0, w=(0.1 if beam else 0.9) / ppc, u=us[s], cell=cells[s],
                            off=offs[s]))
    P = pp.make_params(n, d=(dx, dx, dx), dt=dt, shape_order=O, field_order=fo, alpha=0.55,
                       precision=pp.PP_PREC_FP32_SPLIT, relax_tol=1e-8, relax_max_iter=100,
                       current_scheme=pp.PP_CURRENT_CC if cc else pp.PP_CURRENT_DIRECT,
                       gauss_filter_passes=0 if cc else 5, time_order=torder)
    run = pp.Run(P, species, with_id=False)
    del cells, offs, us
    th = math.radians(74.0)
    dV = dx ** 3
    hist = torch.zeros((steps + 1, 5), dtype=torch.float64, device=dev)
    k1 = torch.fft.fftfreq(g, d=dx, device=dev, dtype=torch.float64) * (2 * math.pi)
    KZ, KY, KX = torch.meshgrid(k1, k1, k1, indexing="ij")
    KK = torch.sqrt(KX * KX + KY * KY + KZ * KZ)
    ang = torch.rad2deg(torch.atan2(torch.sqrt(KX * KX + KY * KY), KZ.abs()))
    band = ((ang >= 60) & (ang <= 80) & (KK >= 1) & (KK <= 8)).to(torch.float64)
    KKs = torch.where(KK > 0, KK, torch.ones_like(KK))
    spec_every = max(1, int(round(0.5 / dt)))
    # wave-number indices 0..kmax, -kmax..-1 as FFT positions (index_select takes no negatives)
    assert 0 <= kmax_index and 2 * kmax_index < g, (kmax_index, g)
    kneg = list(range(0, kmax_index + 1)) + list(range(-kmax_index, 0))
    kidx = torch.tensor([m % g for m in kneg], device=dev)
    bins, bin_t = [], []

    def record(i):
        Ex, Ey, Ez = run.E[0], run.E[1], run.E[2]
        proj = torch.sqrt(Ex * Ex + Ey * Ey) * math.sin(th) + Ez * math.cos(th)
        ezm = Ez.mean(dim=(1, 2))
        hist[i, 0] = 0.5 * dV * (proj * proj).sum()
        hist[i, 1] = 0.5 * dV * (Ez * Ez).sum()
        hist[i, 2] = 0.5 * dV * n[0] * n[1] * (ezm * ezm).sum()
        hist[i, 4] = dV * proj.sum()
        if i % spec_every == 0:
            lon = (torch.fft.fftn(Ex) * KX + torch.fft.fftn(Ey) * KY + torch.fft.fftn(Ez) * KZ) / KKs
            hist[i, 3] = 0.5 * dV / (n[0] * n[1] * n[2]) * (band * lon.abs() ** 2).sum()
            sub = lon.index_select(0, kidx).index_select(1, kidx).index_select(2, kidx)
            bins.append((0.5 * dV / (n[0] * n[1] * n[2]) * sub.abs() ** 2).to(torch.float32))
            bin_t.append(i * dt)
        else:
            hist[i, 3] = float("nan")

    record(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        run.step()
        record(i + 1)
        if progress and (i + 1) % progress == 0:
            torch.cuda.synchronize()
            log(f"[mmi] step {i + 1}/{steps}, W_mmi {hist[i + 1, 0].item():.3e}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    d = run.diagnostics(pp.PP_DIAG_ALL)
    run.close()
    t = np.arange(steps + 1) * dt
    kv = np.array(kneg)
    return t, hist.cpu().numpy(), wall, 4 * npart, d, (np.array(bin_t), kv, torch.stack(bins).cpu().numpy())


def mode_rates(tb, kv, W, dk, t_end, top=12, min_samples=12):
    """Linear growth rates mode by mode.  For every Fourier bin (indices kz, ky, kx from kv,
    energies W [samples, z, y, x] at times tb) the least-squares half log slope of its energy
    over the samples up to t_end (the end of the linear phase) that lie above 30x the bin's
    mean over 1 <= t <= 8 (its noise floor) and below a tenth of its largest value up to
    t_end; bins with fewer than min_samples such samples are left out.  Returns the ``top``
    fastest (one of each +-k pair) with wave vector, |k|, angle to the beam and rate."""
    import numpy as np
    tb = np.asarray(tb, dtype=float)
    L = np.log(np.maximum(W.reshape(len(tb), -1).astype(np.float64), 1e-300))
    floor = L[(tb >= 1.0) & (tb <= 8.0)].mean(axis=0)
    lin = tb <= t_end
    Lmax = np.where(lin[:, None], L, -np.inf).max(axis=0)
    m = lin[:, None] & (L > floor + math.log(30.0)) & (L < Lmax - math.log(10.0))
    n = m.sum(axis=0).astype(float)
    T = tb[:, None]
    St, SL = (m * T).sum(axis=0), (m * L).sum(axis=0)
    Stt, StL = (m * T * T).sum(axis=0), (m * T * L).sum(axis=0)
    den = n * Stt - St * St
    ok = (n >= min_samples) & (den > 0)
    rate = np.where(ok, 0.5 * (n * StL - St * SL) / np.where(ok, den, 1.0), -np.inf)
    KZ, KY, KX = np.meshgrid(kv, kv, kv, indexing="ij")
    KZ, KY, KX = KZ.ravel() * dk, KY.ravel() * dk, KX.ravel() * dk
    kk = np.sqrt(KX * KX + KY * KY + KZ * KZ)
    out, seen = [], set()
    for b in np.argsort(-rate):
        if not np.isfinite(rate[b]):
            break
        if kk[b] == 0:
            continue
        key = tuple(np.round([KZ[b] / dk, KY[b] / dk, KX[b] / dk]).astype(int))
        if tuple(-v for v in key) in seen:
            continue
        seen.add(key)
        ang = math.degrees(math.atan2(math.hypot(KX[b], KY[b]), abs(KZ[b])))
        out.append({"k": [float(KX[b]), float(KY[b]), float(KZ[b])], "abs_k": float(kk[b]), "angle_deg": ang,
                    "rate": float(rate[b]), "samples": int(n[b])})
        if len(out) == top:
            break
    return out


def max_growth(t, w, width):
    """Largest half log slope of the energy w (least squares over windows of the given width)
    between the first time w exceeds 3x its mean over 0 < t <= 2 and the time of its maximum:
    the growth rate of the field amplitude in the steepest part of the growth.  Returns
    (rate, (window start, window end))."""
    import numpy as np
    t = np.asarray(t, dtype=float)
    w = np.asarray(w, dtype=float)
    early = w[(t > 0) & (t <= 2.0)]
    base = early.mean() if early.size else w[w > 0].min()
    above = np.nonzero(w > 3.0 * base)[0]
    i1 = int(np.argmax(w))
    if above.size == 0 or above[0] >= i1:
        return float("nan"), (float("nan"), float("nan"))
    lw = np.log(np.maximum(w, np.finfo(float).tiny))
    best, win = float("nan"), (float("nan"), float("nan"))
    for j in range(int(above[0]), i1):
        k = int(np.searchsorted(t, t[j] + width, side="right"))
        if k > i1 + 1:
            break
        if k - j >= 3:
            r = 0.5 * float(np.polyfit(t[j:k], lw[j:k], 1)[0])
            if not (best >= r):
                best, win = r, (float(t[j]), float(t[k - 1]))
    return best, win


def mmi_rates_fit(t, H, width):
    """Growth rates of the four energies of :func:`run_mmi` (NaN samples skipped): the
    steepest-window rate and the least-squares rate over the whole growth phase."""
    import numpy as np
    out = {}
    for k, col in (("mmi", 0), ("tsi_all_kz", 1), ("tsi", 2), ("mmi_band", 3), ("mmi_linear", 4)):
        ok = np.isfinite(H[:, col])
        # the linear measure grows at the amplitude's rate: square it to fit it as an energy
        w = H[ok, col] ** 2 if col == 4 else H[ok, col]
        rate, window = max_growth(t[ok], w, width)
        _, whole, phase = growth_rate_fit(t[ok], w, width=width)
        out[k] = {"rate": rate, "window": window, "rate_whole_phase": whole, "growth_phase": phase}
    return out


def mmi_bench(args, torch, pp):
    """Relativistic mixed-mode two-stream test: a neutral beam (n_b = 0.1, Lorentz factor 4
    along z) through a neutral background (n_p = 0.9), ion mass 1836 (ions at their
    population's temperature), 128^3 cells of 0.1 c/w_pe (12.8 skin depths), 20 particles per
    cell per species (four species, 167,772,160 particles), cubic weights, 6th-order fields,
    charge-conserving current, FP32 split form; growth rates of the projected-field energies
    against the paper's theory values and its measured values for this scheme."""
    import numpy as np

    from paper_1211_4575_amd import inputs as I
    from paper_1211_4575_amd import inputs_device as ind
    t, H, wall, npart, d, (tb, kv, W) = run_mmi(torch, pp, ind, args.mmi_grid, args.mmi_ppc, args.mmi_steps,
                                                args.mmi_tb, args.mmi_tp, scheme=args.mmi_run, quiet=args.mmi_quiet,
                                                lattice=args.mmi_lattice)
    if args.save_history:
        np.savez(f"{args.save_history}_mmi.npz", t=t, w=H, tb=tb, kv=kv, bins=W)
    theory = I.mmi_rates()
    fits = mmi_rates_fit(t, H, args.mmi_fit_width)
    for k, v in fits.items():
        v["rate_over_theory"] = v["rate"] / (theory["tsi"] if k.startswith("tsi") else theory["mmi"])
        log(f"[mmi] {k}: {v}")
    g = args.mmi_grid
    fits["gamma_tsi_theta0"] = fits["tsi_all_kz"]["rate"]  # the projection at theta_TSI = 0: E_z
    # the linear phase ends when the projected energy reaches 5 % of its largest value
    t_end = float(t[int(np.argmax(H[:, 0] > 0.05 * np.max(H[:, 0])))])
    modes = mode_rates(tb, kv, W, 2 * math.pi / 12.8, t_end)
    for m in modes:
        log(f"[mmi] mode k=({m['k'][0]:+.2f},{m['k'][1]:+.2f},{m['k'][2]:+.2f}) |k|={m['abs_k']:.2f} "
            f"angle {m['angle_deg']:.0f} deg: rate {m['rate']:.4f}")
    out = {"metric": "relativistic mixed-mode two-stream growth rates / theory and paper",
           "theory": theory, "paper_cubic_cc_6th": {"mmi": 0.205, "tsi": 0.088},
           "config": {"grid": [g, g, g], "ppc_per_species": args.mmi_ppc, "particles": npart, "dx": 12.8 / g,
                      "dt": 0.4 * 12.8 / g, "steps": args.mmi_steps, "T_b": args.mmi_tb, "T_p": args.mmi_tp,
                      "run": args.mmi_run, "field_order": MMI_SCHEMES[args.mmi_run][0],
                      "shape_order": MMI_SCHEMES[args.mmi_run][1], "charge_conserving": MMI_SCHEMES[args.mmi_run][2],
                      "time_order": MMI_SCHEMES[args.mmi_run][3], "quiet_start": bool(args.mmi_quiet),
                      "lattice": args.mmi_lattice},
           "updates_per_s": npart * args.mmi_steps / wall, "wall_s": wall,
           "final_gauss_rel": d.gauss_max / d.rho_ref, "flags": d.flags, "linear_phase_end": t_end,
           "fastest_modes": modes, **fits}
    print(json.dumps(out), flush=True)
    return 0


def kh_tile_unevenness(run, torch, pp, n, t=(8, 8)):
    """Largest over mean particle count of the 8x8x1 tiles (all species), from the device
    arrays of the current positions."""
    nt0 = (n[0] + t[0] - 1) // t[0]
    ntiles = nt0 * ((n[1] + t[1] - 1) // t[1])
    counts = torch.zeros(ntiles, dtype=torch.int64, device=run.E.device)
    for s in range(len(run.species)):
        P = pp.pp_get_particles(run.handle, s)
        cell = run._wrap_ptr(P.cell, P.n, None).to(torch.int64)
        i, j = cell % n[0], (cell // n[0]) % n[1]
        counts += torch.bincount((i // t[0]) + nt0 * (j // t[1]), minlength=ntiles)
    return float(counts.max()) / float(counts.double().mean())


def kh_long_run(run, torch, pp, n, npart, steps, window=50):
    """The shear-flow run over ``steps`` steps: whole-step rate over windows at the start, the
    middle and the end, tile unevenness, normalised Gauss residual and field energies there."""
    out = []
    marks = (0, steps // 2, steps - window)
    done = 0
    for m in marks:
        while done < m:
            run.step()
            done += 1
            if done % 500 == 0:
                torch.cuda.synchronize()
                log(f"[kh] step {done}/{steps}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(window):
            run.step()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        done += window
        d = run.diagnostics(pp.PP_DIAG_RHO | pp.PP_DIAG_FIELDS)
        rec = dict(steps=[m, m + window], updates_per_s=npart * window / wall, ms_per_step=1e3 * wall / window,
                   tile_max_over_mean=kh_tile_unevenness(run, torch, pp, n), gauss_rel=d.gauss_max / d.rho_ref,
                   field_E=d.field_E, field_B=d.field_B, flags=d.flags)
        log(f"[kh] {rec}")
        out.append(rec)
    return out


def kh_bench(args, torch, pp):
    """Kelvin-Helmholtz shear layers: 1024x512x1 cells, electrons and ions (mass ratio 25),
    64 particles per cell each (67,108,864 particles), bulk flows +-0.2c, u_th = 0.02c,
    cubic weights, 6th-order fields, dt 0.4: whole-step throughput of the FP32 split form on
    the flat (8x8x1) tile path, and of the FP64 plain form."""
    from paper_1211_4575_amd import inputs_device as ind
    n, ppc = (1024, 512, 1), 64
    npart = n[0] * n[1] * n[2] * ppc
    dev = torch.device("cuda:0")
    res = {}
    for split in ((True, False) if not args.no_fp64 else (True,)):
        rt = torch.float32 if split else torch.float64
        cells = [torch.empty(npart, dtype=torch.int32, device=dev) for _ in range(2)] if split else None
        offs = [torch.empty((3, npart), dtype=rt, device=dev) for _ in range(2)]
        us = [torch.empty((3, npart), dtype=rt, device=dev) for _ in range(2)]
        ind.kelvin_helmholtz(SEED, n, 0, npart, 0.2, 8.0, 0.02, ind.split_mode(split, 3), cells,
                             [[o[d] for d in range(3)] for o in offs], [[u[d] for d in range(3)] for u in us],
                             torch.cuda.current_stream().cuda_stream)
        species = []
        for s, (q, m) in enumerate(((-1.0, 1.0), (1.0, 25.0))):
            sp = dict(q=q, m=m, w=1.0 / ppc, u=us[s])
            sp.update(dict(cell=cells[s], off=offs[s]) if split else dict(pos=offs[s]))
            species.append(sp)
        P = pp.make_params(n, shape_order=3, field_order=6, dt=0.4, alpha=0.55,
                           precision=pp.PP_PREC_FP32_SPLIT if split else pp.PP_PREC_FP64,
                           relax_tol=1e-8 if split else 1e-14, relax_max_iter=100)
        run = pp.Run(P, species, with_id=False)
        del cells, offs, us
        key = "fp32_split" if split else "fp64_plain"
        if split and args.kh_steps > 0:
            res["long_run"] = kh_long_run(run, torch, pp, n, 2 * npart, args.kh_steps)
        steps = args.steps if split else max(1, args.fp64_steps)
        wall, gpd_ms = time_steps(run, torch, steps, args.warmup if split else 1)
        d = run.diagnostics(pp.PP_DIAG_MOMENTS | pp.PP_DIAG_FIELDS)
        res[key] = dict(updates_per_s=2 * npart * steps / wall, ms_per_step=1e3 * wall / steps,
                        gpd_updates_per_s=2 * npart / (gpd_ms * 1e-3), flags=d.flags)
        log(f"[kh] {key}: {res[key]}")
        run.close()
        del run
        torch.cuda.empty_cache()
    out = {"metric": "particle updates/s (gather+push+deposit) FP32 vs FP64; ensemble p50/p99",
           "value": res["fp32_split"]["updates_per_s"], "unit": "particle updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["fp32_split"]["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "Kelvin-Helmholtz 1024x512x1, 64 ppc/species, mass ratio 25, flows +-0.2c, "
                                  "cubic weights, 6th-order fields, FP32 split positions (flat 8x8x1 tiles)",
                      "particles": 2 * npart, "results": res}}
    print(json.dumps(out), flush=True)
    return 0


def serving_leg(torch, pp, count=32, rate=4.0, slots=64, mem_gib=160.0, sample=4, no_fp64=False):
    """A bounded serving run for the default benchmark line: `count` requests of the serving
    ensemble (two-stream runs on 32^3 / 64x32x32 / 128x16x16 grids, 8-64 particles per cell per
    beam, 200-2000 steps) arriving as a Poisson stream at `rate` per second, served by continuous
    batching (FP32 split form).  Beside it, the `sample` requests with the fewest updates are run
    one at a time, each whole, in the plain FP64 form and in the FP32 split form (measured, not
    modelled), and the per-class model of the one-at-a-time service (measured steps of each
    grid/lattice class x the request's steps) is checked against those runs and used for the
    FIFO latency of the whole stream."""
    from paper_1211_4575_amd import inputs as I
    from paper_1211_4575_amd import serve as S
    reqs = I.serving_requests(count=count, rate=rate, seed=SEED)
    be = S.DeviceBackend(max_slots=slots)
    try:
        sched = S.Scheduler(be, mem_budget=int(mem_gib * (1 << 30)), max_slots=slots)
        res = sched.run(reqs)
        out = {"requests": count, "rate_per_s": rate, "batched_fp32": S.summarize(res, t_first=0.0),
               "peak_members": sched.peak_members}
        log(f"[serve-leg] batched: {out['batched_fp32']}")
        small = sorted(reqs, key=lambda r: r.updates)[:sample]
        measured = []
        for q in small:
            row = {"rid": q.rid, "grid": list(q.n), "ppc_per_beam": q.ppc, "steps": q.steps, "updates": q.updates}
            for key, split in (("fp32_split_s", True), ("fp64_plain_s", False)):
                if not split and no_fp64:
                    continue
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                run = be.make_run(q, split=split)
                for _ in range(q.steps):
                    run.step()
                torch.cuda.synchronize()
                row[key] = time.perf_counter() - t0
                run.close()
            batched = next(r for r in res if r.rid == q.rid)
            row["batched_latency_s"] = batched.latency
            measured.append(row)
            log(f"[serve-leg] alone: {row}")
        out["alone_measured"] = measured
        for name, split in (("fp64_plain_one_at_a_time", False), ("fp32_split_one_at_a_time", True)):
            if not split and no_fp64:
                continue
            r1, per_class = S.one_at_a_time_reference(be, reqs, split=split, steps=3)
            s1 = S.summarize(r1, t_first=0.0)
            model = {r.rid: (r.done - r.admitted) for r in r1}
            key = "fp32_split_s" if split else "fp64_plain_s"
            s1["model_over_measured"] = [round(model[m["rid"]] / m[key], 3) for m in measured]
            s1["kind"] = ("FIFO over the same arrivals; service time = measured per-step time of the request's "
                          "grid/lattice class x its steps + set-up")
            out[name] = s1
            log(f"[serve-leg] {name}: {s1}")
        if "fp64_plain_one_at_a_time" in out and out["batched_fp32"].get("updates_per_s"):
            out["speedup_vs_fp64_one_at_a_time"] = (out["batched_fp32"]["updates_per_s"] /
                                                   out["fp64_plain_one_at_a_time"]["updates_per_s"])
        return out
    finally:
        be.close()
        torch.cuda.empty_cache()


def serving_bench(args, torch, pp):
    """The serving ensemble: a Poisson stream of two-stream requests (grids 32^3, 64x32x32,
    128x16x16; 8-64 particles per cell per beam; beam speed 0.1-0.5 c; 200-2000 steps), served
    by continuous batching of FP32 split-precision runs; p50/p99 completion latency and
    aggregate updates/s, beside the same requests served one at a time (FP64 plain form and
    FP32 split form, from measured per-step times)."""
    from paper_1211_4575_amd import inputs as I
    from paper_1211_4575_amd import serve as S

    reqs = I.serving_requests(count=args.requests, rate=args.rate, seed=SEED)
    be = S.DeviceBackend(max_slots=args.slots)
    log(f"[serve] {len(reqs)} requests, rate {args.rate}/s, {sum(r.updates for r in reqs):.3e} updates, "
        f"budget {args.mem_gib} GiB, {args.slots} slots")
    done = []

    def progress(r, members):
        done.append(r)
        if len(done) % 8 == 0 or len(done) == len(reqs):
            log(f"[serve] {len(done)}/{len(reqs)} done at t={r.done:.1f} s (request {r.rid}: latency "
                f"{r.latency:.2f} s, {r.status}), {members} runs in the batch")

    sched = S.Scheduler(be, mem_budget=int(args.mem_gib * (1 << 30)), max_slots=args.slots, on_complete=progress)
    t0 = time.perf_counter()
    res = sched.run(reqs)
    wall = time.perf_counter() - t0
    summ = S.summarize(res, t_first=0.0)
    log(f"[serve] batched: {summ}, wall {wall:.1f} s, peak members {sched.peak_members}, "
        f"peak {sched.peak_bytes / 2**30:.1f} GiB, {sched.batch_steps} batch steps")
    refs = {}
    for name, split in (("fp64_plain_one_at_a_time", False), ("fp32_split_one_at_a_time", True)):
        if split is False and args.no_fp64:
            continue
        r1, per_class = S.one_at_a_time_reference(be, reqs, split=split, steps=args.ref_steps)
        s1 = S.summarize(r1, t_first=0.0)
        s1["ms_per_step_by_class"] = per_class
        s1["kind"] = "measured per-step time of each grid/lattice class x steps + set-up, FIFO over the same arrivals"
        refs[name] = s1
        log(f"[serve] {name}: {s1}")
    be.close()
    fails = [r.rid for r in res if r.status != "ok"]
    out = {
        "metric": "particle updates/s (gather+push+deposit) FP32 vs FP64; ensemble p50/p99",
        "value": summ.get("updates_per_s"),
        "unit": "particle updates/s",
        "n_gpus": 1,
        "steps": sched.batch_steps,
        "warmup": 0,
        "ms_per_step": 1e3 * summ.get("makespan_s", math.nan) / max(sched.batch_steps, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"serving ensemble: {len(reqs)} two-stream requests, Poisson arrivals at {args.rate}/s, "
                               f"grids 32^3/64x32x32/128x16x16, 8-64 ppc per beam, 200-2000 steps, cubic weights, "
                               f"6th-order fields, FP32 split, continuous batching",
                   "p50_s": summ.get("p50_s"), "p99_s": summ.get("p99_s"), "makespan_s": summ.get("makespan_s"),
                   "completed": summ.get("completed"), "failed": fails, "peak_members": sched.peak_members,
                   "peak_gib": round(sched.peak_bytes / 2**30, 2), "mem_budget_gib": args.mem_gib,
                   "slots": args.slots, "references": refs,
                   "speedup_vs_fp64_one_at_a_time": (summ["updates_per_s"] / refs["fp64_plain_one_at_a_time"]["updates_per_s"])
                   if "fp64_plain_one_at_a_time" in refs and summ.get("updates_per_s") else None},
    }
    print(json.dumps(out), flush=True)
    return 0


def lds_probe():
    """Compile bench_lds_rates.hip (beside this file) for gfx950 and run it: the clocks per
    wavefront instruction of the LDS and VALU instructions the particle kernel's cost model uses."""
    import subprocess
    src = os.path.join(ROOT, "bench_lds_rates.hip")
    exe = os.path.join(ROOT, "_build", "bench_lds_rates")
    os.makedirs(os.path.dirname(exe), exist_ok=True)
    subprocess.check_call([os.environ.get("HIPCC", "/opt/rocm/bin/hipcc"), "-O3", "-std=c++17", "--offload-arch=gfx950",
                           "-munsafe-fp-atomics", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", src,
                           "-o", exe], stderr=subprocess.DEVNULL)
    return subprocess.call([exe])


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--ppc", type=int, default=32)
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="leave out the bounded serving leg")
    ap.add_argument("--serving-requests", type=int, default=32, help="requests of the bounded serving leg")
    ap.add_argument("--rad-tau", type=float, default=0.0, help="radiative cooling constant (0: off)")
    ap.add_argument("--current", choices=("cc", "direct"), default="cc",
                    help="current scheme: charge-conserving (default) or direct")
    ap.add_argument("--gauss-passes", type=int, default=0, help="Gauss-law filter passes per step")
    ap.add_argument("--time-order", type=int, choices=(2, 4), default=2,
                    help="2: leapfrog; 4: fourth-order composition (three substeps per step)")
    ap.add_argument("--calib-copy-gib", type=float, default=0.0,
                    help="also run a plain device copy of this size (counter calibration)")
    ap.add_argument("--workload", choices=("pair_mj", "serving", "two_stream", "kh", "mmi"), default="pair_mj")
    ap.add_argument("--mmi-grid", type=int, default=128, help="mmi: cells per axis (box 12.8 skin depths)")
    ap.add_argument("--mmi-ppc", type=int, default=20, help="mmi: particles per cell per species")
    ap.add_argument("--mmi-steps", type=int, default=1500, help="mmi: steps")
    ap.add_argument("--mmi-fit-width", type=float, default=6.0, help="mmi: fit window (1/w_pe)")
    ap.add_argument("--mmi-quiet", action="store_true",
                    help="mmi: quiet start (particle pairs with opposite thermal velocities)")
    ap.add_argument("--mmi-lattice", type=int, nargs=3, default=None, metavar=("PX", "PY", "PZ"),
                    help="mmi: positions on a regular lattice of PX*PY*PZ (= ppc) points per cell")
    ap.add_argument("--mmi-run", type=int, choices=sorted(MMI_SCHEMES), default=5,
                    help="mmi: scheme of the paper's comparison (1-4 direct current + filter, 5 charge-conserving, "
                         "6 with fourth-order time integration)")
    ap.add_argument("--mmi-tb", type=float, default=1e-4,
                    help="mmi: beam temperature (m_e c^2); the default reads the paper's 0.01 as u_th")
    ap.add_argument("--mmi-tp", type=float, default=0.01,
                    help="mmi: background temperature (m_e c^2); the default reads the paper's 0.1 as u_th")
    ap.add_argument("--grid-x", type=int, default=128, help="two-stream: cells along the beams")
    ap.add_argument("--kh-steps", type=int, default=0,
                    help="kh: also run this many steps, timing windows at the start, middle and end")
    ap.add_argument("--ts-steps", type=int, default=2000, help="two-stream: steps")
    ap.add_argument("--save-history", default="", help="two-stream: save the E_x energy history to PATH_<form>.npz")
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--rate", type=float, default=2.0, help="serving: mean arrivals per second")
    ap.add_argument("--slots", type=int, default=64, help="serving: most runs in the batch")
    ap.add_argument("--mem-gib", type=float, default=160.0, help="serving: device memory budget for runs")
    ap.add_argument("--ref-steps", type=int, default=3, help="serving: timed steps per class for the references")
    ap.add_argument("--cpu-plan", action="store_true",
                    help="time the CPU oracle on the whole baseline plan (one core and all cores) and exit")
    ap.add_argument("--counter-summary", nargs="+", default=None, metavar="DIR",
                    help="write profiles/k_gpd32_pair_mj_256_counters.md from these rocprofv3 --pmc folders and exit")
    ap.add_argument("--counter-cmd", action="append", default=[], help="command line recorded in the summary")
    ap.add_argument("--stats-summary", default=None, metavar="DIR",
                    help="write profiles/k_gpd32_pair_mj_256_kernel_stats.md from this rocprofv3 --stats folder and exit")
    ap.add_argument("--lds-probe", action="store_true",
                    help="build and run the LDS / VALU instruction-rate probe (bench_lds_rates.hip) and exit")
    args = ap.parse_args(argv)
    if args.lds_probe:
        return lds_probe()
    if args.stats_summary:
        n = args.grid
        print(stats_summary(args.stats_summary, os.path.join(ROOT, "profiles", "k_gpd32_pair_mj_256_kernel_stats.md"),
                            2 * n * n * n * args.ppc, " ".join(args.counter_cmd)))
        return 0
    if args.counter_summary:
        n = args.grid
        print(counter_summary(args.counter_summary, os.path.join(ROOT, "profiles", "k_gpd32_pair_mj_256_counters.md"),
                              2 * n * n * n * args.ppc, args.counter_cmd))
        return 0
    if args.cpu_plan:
        return cpu_plan()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): sharding the path over "
              f"GPUs (sub-boxes of whole tiles with halo exchange) is not built.", file=sys.stderr)
        return 2

    import torch

    from paper_1211_4575_amd import inputs_device as ind
    from paper_1211_4575_amd import pp

    if args.workload == "serving":
        return serving_bench(args, torch, pp)
    if args.workload == "two_stream":
        return two_stream_bench(args, torch, pp)
    if args.workload == "kh":
        return kh_bench(args, torch, pp)
    if args.workload == "mmi":
        return mmi_bench(args, torch, pp)

    if args.calib_copy_gib > 0:
        nb = int(args.calib_copy_gib * (1 << 30))
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        # the same bytes through an ordinary elementwise kernel (plain vector loads and stores)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy and elementwise pass of {nb} bytes each")
        del src, dst
        torch.cuda.empty_cache()

    n = (args.grid, args.grid, args.grid)
    log(f"[bench] FP32 split: generating {n} x {args.ppc} ppc x 2 species on the device")
    scheme = pp.PP_CURRENT_DIRECT if args.current == "direct" else pp.PP_CURRENT_CC
    run, npart = make_pair_mj_run(pp, ind, torch, n, args.ppc, 1.0, split=True, rad_tau=args.rad_tau,
                                  current_scheme=scheme, gauss_passes=args.gauss_passes, time_order=args.time_order)
    npart *= 2  # electrons and positrons
    log(f"[bench] FP32 split: {npart} particles; warmup {args.warmup}, timing {args.steps} steps")
    wall, gpd_ms = time_steps(run, torch, args.steps, args.warmup)
    ms_step = 1e3 * wall / args.steps
    value = npart * args.steps / wall
    gpd_rate = npart / (gpd_ms * 1e-3)
    log(f"[bench] FP32: {ms_step:.2f} ms/step, gpd kernel {gpd_ms:.2f} ms -> {gpd_rate:.3e} updates/s")
    # per-step charge conservation and Gauss residual (FP64), outside the timed region
    run.diagnostics(pp.PP_DIAG_RHO)
    run.step()
    torch.cuda.synchronize()
    t_diag = time.perf_counter()
    dg = run.diagnostics(pp.PP_DIAG_ALL)  # returns after the device has finished
    t_diag = time.perf_counter() - t_diag
    diag32 = dict(cc_rel=dg.cc_max / dg.rho_ref, gauss_rel=dg.gauss_max / dg.rho_ref, flags=dg.flags,
                  relax_sweeps=dg.relax_iters, relax_bound=dg.relax_resid, diag_all_ms=round(1e3 * t_diag, 2))
    log(f"[bench] FP32 diagnostics {diag32}")
    run.close()
    del run
    torch.cuda.empty_cache()

    fp64 = None
    if not args.no_fp64:
        log(f"[bench] FP64 plain: generating")
        run, _ = make_pair_mj_run(pp, ind, torch, n, args.ppc, 1.0, split=False, rad_tau=args.rad_tau,
                                  current_scheme=scheme, gauss_passes=args.gauss_passes, time_order=args.time_order)
        log(f"[bench] FP64 plain: warmup 1, timing {args.fp64_steps} steps")
        wall64, gpd64_ms = time_steps(run, torch, args.fp64_steps, 1)
        fp64 = dict(form="plain FP64: untiled, one thread per particle, every current contribution a global "
                         "FP64 atomic (the ratio measures the tiled split design, not the precision alone)",
                    value=npart * args.fp64_steps / wall64, ms_per_step=1e3 * wall64 / args.fp64_steps,
                    gpd_updates_per_s=npart / (gpd64_ms * 1e-3), gpd_ms=gpd64_ms)
        # per-step charge conservation and Gauss residual of the FP64 form, outside the timed region
        run.diagnostics(pp.PP_DIAG_RHO)
        run.step()
        dg = run.diagnostics(pp.PP_DIAG_ALL)
        fp64["diagnostics"] = dict(cc_rel=dg.cc_max / dg.rho_ref, gauss_rel=dg.gauss_max / dg.rho_ref, flags=dg.flags)
        log(f"[bench] FP64 plain {fp64}")
        run.close()
        del run
        torch.cuda.empty_cache()

    roofline = kernel_roofline(npart, gpd_ms, direct=args.current == "direct")

    serving = None
    if not args.no_serving:
        log(f"[bench] serving leg: {args.serving_requests} requests")
        serving = serving_leg(torch, pp, count=args.serving_requests, no_fp64=args.no_fp64)

    cpu = None
    if not args.no_cpu:
        log("[bench] CPU baseline (oracle, bounded sample)")
        cpu = cpu_baseline()
        log(f"[bench] CPU {cpu}")

    out = {
        "metric": "particle updates/s (gather+push+deposit) FP32 vs FP64; ensemble p50/p99",
        "value": value,
        "unit": "particle updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"pair plasma {n[0]}x{n[1]}x{n[2]}, {args.ppc} ppc/species, Maxwell-Juttner kT=mc^2, "
                               f"cubic weights, 6th-order fields, FP32 split positions",
                   "particles": npart, "step": "gather/push/deposit + line solve + sort + field step", "rad_tau": args.rad_tau,
                   "current": args.current, "gauss_passes": args.gauss_passes, "time_order": args.time_order,
                   "gpd_updates_per_s": gpd_rate, "fp64_plain": fp64,
                   "fp32_over_fp64": (value / fp64["value"]) if fp64 else None, "diagnostics": diag32},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
