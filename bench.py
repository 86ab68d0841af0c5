"""Benchmark of the mDPD timestep on one MI355X.

Workload: periodic bulk mDPD liquid, 56 x 56 x 56 box at number density 6
(1,053,696 particles), A = -40, B = 25, r_c = 1, r_d = 0.75, gamma = 4.5,
kT = 1, dt = 0.01, uniform-random start, Maxwell velocities (seed 0).  One
"step" is one full timestep of the hot path: bin + sort, neighbour list,
density pass, force pass with the velocity-Verlet epilogue.

Prints ONE JSON line: particle-steps/s of the FP32-forces form (value) next
to the all-FP64 form, timed over `--steps` steps after `--relax` untimed
steps from the random start and `--warmup` more, with kernel timing off; the
per-kernel HIP-event times come from a separate pass.  `roofline` is the
kernel class with the most time per step, priced on its share of the step's
algorithmic VALU work (pair geometry for the neighbour list, noise and force
terms plus the velocity-Verlet update for the force pass, the weights for the
density pass); the step's own VALU and HBM fractions use the whole count and
the algorithmic bytes (density 29 B, force 105 B, 142 B per re-sort).
Measured traffic and instruction counts appear as overhead ratios.
`cpu_baseline` is the FP64 oracle timed on the host's cores on a bounded
sample.

    python bench.py [--gpus 1] [--steps 1000] [--warmup 100] [--relax 300] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks: HBM3E 8 TB/s; VALU 256 CUs x 64 lanes x 2.4 GHz
# = 39.32 T lane-instructions/s (one FP32/FP64/int32 op per lane per clock,
# no packed math; FP64 FMA is full rate on CDNA4: 78.6 TFLOP/s = 2 x 39.3 T).
PEAK_HBM_GBS = 8000.0
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12

# Algorithmic work of one timestep (the count of the survey's measurement
# section), per unique pair within r_c: pair geometry with the square root
# 15 ops, Threefry-2x32-20 noise 75, the force terms and their accumulation
# 30; per unique pair within r_d the density weight 16; per particle the
# velocity-Verlet update 20.  The geometry is the neighbour list's share,
# the noise and force terms the force kernel's, so that the kernel shares add
# up to the step's count (about 1.6 k ops per particle-step at density 6).
OPS_PAIR_GEOMETRY = 15
OPS_PAIR_FORCE = 105
OPS_DENSITY_PAIR = 16
OPS_VV_PARTICLE = 20
# Algorithmic HBM bytes per particle (every array touched once per pass):
# density pass reads x 24 and type/flags 1 and writes rho 4; force pass
# reads x 24, v_half 24, rho 4, type 1, id 4 and writes x' 24, v_half' 24;
# a re-sort moves the state once (142 B).  The FP64 form's rho is 8 bytes
# (+4 in each pass).  The neighbour list is no algorithmic traffic: its
# share is the read of x (24 B).
BYTES_DENSITY = {"fp32_forces": 29, "fp64": 33}
BYTES_FORCE = {"fp32_forces": 105, "fp64": 109}
BYTES_RESORT = 142
BYTES_LIST = 24
# Measured overheads of the FP32-form kernels on this workload (rocprofv3 on
# the same command as bench.py's default; profiles/mdpd_step_bulk56_n1053696.md):
# HBM traffic from FETCH_SIZE / WRITE_SIZE scaled by a plain 256 MiB copy
# (x2.000 reads, x1.000 writes) and VALU instructions per dispatch
# (SQ_INSTS_VALU, wave instructions).  Valid for the kernels as profiled;
# they are re-measured whenever a kernel changes.
PROFILED = {
    "nlist": {"read": 79714304, "write": 181342208, "valu_wave_instr": 120.9e6},
    "force": {"read": 300464128, "write": 101422080, "valu_wave_instr": 75.7e6},
    "density": {"read": 126672896, "write": 37933056, "valu_wave_instr": 14.2e6},
}

def list_candidates(x, box, rc=1.0):
    """Number of (i, j != i) candidate pairs the cell-list search tests: every
    particle of the 27 cells around (and including) i's cell, cells of edge
    L / floor(L / r_c) per axis, periodic."""
    nc = [int(np.floor(L / rc)) for L in box]
    c = [np.minimum((x[:, a] * nc[a] / box[a]).astype(np.int64), nc[a] - 1) for a in range(3)]
    cnt = np.zeros(nc, np.int64)
    np.add.at(cnt, (c[0], c[1], c[2]), 1)
    stencil = np.zeros_like(cnt)
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                stencil += np.roll(cnt, (dx, dy, dz), axis=(0, 1, 2))
    return int((cnt * stencil).sum()) - x.shape[0]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--L", type=float, default=56.0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-steps", type=int, default=12,
                    help="oracle steps of the CPU baseline (about 10 s on 16 cores)")
    ap.add_argument("--brute-steps", type=int, default=10,
                    help="oracle steps of the O(N^2) CPU legs on the 6,000-particle box")
    ap.add_argument("--relax", type=int, default=300,
                    help="untimed steps from the uniform-random start before the warm-up")
    ap.add_argument("--lanes", type=str, default="", help="n,d,f lanes per particle")
    ap.add_argument("--forms", type=str, default="fp32_forces,fp64,fp32_forces_skin",
                    help="fp32_forces (the headline), fp64, fp32_forces_skin (FP32 with a list skin)")
    ap.add_argument("--skin", type=float, default=0.3, help="list skin of the fp32_forces_skin form")
    ap.add_argument("--replicas", type=int, default=256, help="replicas of the batched workload (0: skip)")
    ap.add_argument("--no-walls", action="store_true", help="skip the walled channel and rock workloads")
    ap.add_argument("--no-small", action="store_true", help="skip the 6,000-particle eager vs graph workload")
    ap.add_argument("--walled", type=str, default="channel,rock,ring_cells",
                    help="walled workloads to run (comma list of channel, rock, ring_cells)")
    ap.add_argument("--walled-only", action="store_true",
                    help="run only the walled workloads and print their results (for profiling them)")
    ap.add_argument("--adj-steps", type=int, default=100, help="steps of the batched forward + adjoint")
    ap.add_argument("--adj-every", type=int, default=10, help="checkpoint spacing of the adjoint")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MiB",
                    help="only run a plain device copy of this size 5 times (counter scaling)")
    return ap.parse_args()


def copy_calibration(mib):
    """A plain copy kernel of known size: reads and writes mib MiB per launch."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_per_launch": n * 4, "launches": 5}), flush=True)


def run_form(mdpd, w, precision, steps, warmup, relax, stream, lanes, skin=0.0):
    """Relax the uniform-random start (untimed), warm up, time `steps` steps
    with kernel timing off, then take the per-kernel HIP-event times over a
    separate pass of min(steps, 200) steps."""
    import torch
    s = mdpd.System(w, precision=precision, stream=stream, device_inputs=True, skin=skin)
    if lanes:
        for k, v in enumerate(lanes):
            s.set_lanes(k, v)
    s.step(relax + warmup)
    torch.cuda.synchronize()
    obs0 = s.observables()
    b0 = s.list_builds()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    builds = s.list_builds() - b0
    obs = s.observables()
    kt_steps = min(steps, 200)
    mdpd.mdpd_set_kernel_timing(s.h, True)
    for k in range(len(mdpd.KERNELS)):
        mdpd.mdpd_read_kernel_timing(s.h, k)  # reset
    s.step(kt_steps)
    torch.cuda.synchronize()
    ktime = {name: mdpd.mdpd_read_kernel_timing(s.h, k) for k, name in enumerate(mdpd.KERNELS)}
    mdpd.mdpd_set_kernel_timing(s.h, False)
    cnt_c, _ = s.neighbors(w.rc)
    cnt_d, _ = s.neighbors(w.rd)
    x, _, _ = s.state()
    s.close()
    return dict(sec=t1 - t0, ktime=ktime, kt_steps=kt_steps, obs=obs, kT_start=obs0["kT"], skin=skin,
                builds_per_step=builds / max(steps, 1),
                pairs_c=int(cnt_c.sum()) // 2, pairs_d=int(cnt_d.sum()) // 2,
                candidates=list_candidates(np.asarray(x), w.box, w.rc))


def run_batch(mdpd, W, nrep, steps, every):
    """Batched replicas (edges U[8, 12], A ~ U[-50, -30], B ~ U[20, 30], FP32
    forces): forward throughput, then a recording of `steps` steps with a
    checkpoint every `every` and the adjoint of the mean density and pressure
    (time-averaged) with respect to A, B, gamma of every replica."""
    import torch
    reps = W.replicas(count=nrep, lo=8.0, hi=12.0, seed=0)
    n = sum(r.n for r in reps)
    b = mdpd.Batch(reps, precision=mdpd.FP32_FORCES, device_inputs=True)
    b.step(10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    fwd = time.perf_counter() - t0
    # the same forward steps after the autotuner, replayed as a HIP graph
    tuned = [int(v) for v in b.autotune(steps=5)]
    b.set_graph(True)
    b.step(10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    fwd_tg = time.perf_counter() - t0
    b.close()
    # adjoint: a warm-up cycle allocates the checkpoints and the tape, then
    # the state at step 0 is restored and the timed cycle runs
    a = mdpd.Batch(reps, precision=mdpd.FP32_FORCES, device_inputs=True)
    ck0 = mdpd.mdpd_save_checkpoint(a.h)
    wts = np.tile([1.0, 0.05, 0.0], (nrep, 1))
    a.forward_record(steps, every=every, average=True)
    a.backward(wts)
    mdpd.mdpd_load_checkpoint(a.h, ck0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = a.forward_record(steps, every=every, average=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g = a.backward(wts)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    a.close()
    return {"workload": f"{nrep} replicas, periodic boxes with edges U[8, 12] at density 6, "
                        f"A ~ U[-50, -30], B ~ U[20, 30], FP32 forces",
            "replicas": nrep, "particles": n, "steps": steps, "checkpoint_every": every,
            "forward_particle_steps_per_s": n * steps / fwd, "forward_ms_per_step": fwd * 1e3 / steps,
            "tuned_graph_forward_ms_per_step": fwd_tg * 1e3 / steps, "tuned_lanes": tuned,
            "tuned_graph_particle_steps_per_s": n * steps / fwd_tg,
            "record_s": t1 - t0, "backward_s": t2 - t1, "forward_s": fwd,
            "adjoint_over_forward": (t2 - t1) / fwd,
            "record_plus_adjoint_over_forward": (t2 - t0) / fwd,
            "loss_mean_rho_r0": float(loss[0][0]), "dA_r0": float(g["dA"][0][0, 0])}


def run_small(mdpd, W, steps):
    """The 6,000-particle box (L = 10): latency-bound, so eager launches,
    a replayed HIP graph, and a graph after the autotuner (list split, lanes
    of the density and force passes) are compared."""
    import torch
    w = W.bulk(L=10.0, seed=0)
    out = {"workload": "bulk mDPD liquid, periodic 10^3 box, 6000 particles", "particles": w.n, "steps": steps}
    for mode in ("eager", "graph", "tuned_graph"):
        s = mdpd.System(w, precision=mdpd.FP32_FORCES, device_inputs=True)
        if mode == "tuned_graph":
            out["tuned_lanes"] = [int(v) for v in s.autotune(steps=20)]
        s.set_graph(mode != "eager")
        s.step(20)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        s.close()
        out[f"{mode}_us_per_step"] = sec * 1e6 / steps
        out[f"{mode}_particle_steps_per_s"] = w.n * steps / sec
    return out


def run_walled(mdpd, w, steps, warmup):
    """A walled workload (frozen wall particles, boundary-volume-fraction
    corrector, body force), FP32 forces: step time and corrector activity over
    `steps` timed steps after `warmup` untimed ones (the rock's random filling
    settles, kT 1.3 -> 1.01, within its first 300 steps)."""
    import torch
    s = mdpd.System(w, precision=mdpd.FP32_FORCES, device_inputs=True)
    s.step(warmup)
    c0 = s.observables()["ncorr_total"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    o = s.observables()
    s.close()
    nf = int(w.n - int(np.asarray(w.frozen).sum()))
    return {"particles": w.n, "fluid": nf, "box": list(w.box), "steps": steps,
            "ms_per_step": sec * 1e3 / steps, "particle_steps_per_s": w.n * steps / sec,
            "fluid_particle_steps_per_s": nf * steps / sec, "kT": o["kT"],
            "mean_v": [m / max(nf, 1) for m in o["momentum"]],
            "warmup": warmup, "corrections_per_step": (o["ncorr_total"] - c0) / steps}


WALLED = {
    "channel": (lambda W: W.channel(), 200, 20,
                "Poiseuille channel 64 x 32 x 64, frozen walls of thickness 2, g_x = 0.02"),
    "rock": (lambda W: W.rock(), 100, 300,
             "synthetic rock, 128^3 Gaussian-random-field mask, porosity 0.3, g_x = 0.01"),
    "ring_cells": (lambda W: W.ring_cells(n=23, layers=1), 200, 20,
                   "manufactured homogeneous porous medium (ring cells 16 x 2 x 16, solid density 8, "
                   "fluid 6.2, g_z = 0.02): 23 x 23 cells of the paper's thickness 2"),
}


def run_walled_set(mdpd, W, names):
    out = {}
    for k in [v for v in names.split(",") if v]:
        make, steps, warmup, desc = WALLED[k]
        out[k] = run_walled(mdpd, make(W), steps, warmup)
        out[k]["workload"] = desc
        v = out[k]
        print(f"# {k}: {v['particles']} particles ({v['fluid']} fluid), {v['ms_per_step']:.3f} ms/step, "
              f"{v['corrections_per_step']:.1f} corrections/step", file=sys.stderr, flush=True)
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


def cpu_baseline(w, W, nsteps, brute_steps):
    """The FP64 oracle on the host's cores.  value: its linked-cell search on
    the benchmark's own workload (the fair O(N) CPU baseline); legs: the
    brute-force O(N^2) search (the oracle's definition) on the 6,000-particle
    box on one core and on all cores, and that rate carried to the 1M box by
    N^2 scaling (extrapolated, not run: one such step would take minutes)."""
    import oracle
    cores = oracle.num_threads()
    p = oracle.make_params(**w.param_kwargs(), search=1)
    t0 = time.perf_counter()
    o = oracle.System(p, w.x, w.v)
    t1 = time.perf_counter()
    o.step(nsteps)
    t2 = time.perf_counter()
    del o
    out = dict(value=w.n * nsteps / (t2 - t1), unit="particle-steps/s", cores=cores, kind="oracle",
               cpu_model=cpu_model(),
               sample=f"{nsteps} steps of the same {w.n}-particle workload with the oracle's "
                      f"linked-cell search (FP64, OpenMP over particles), after a "
                      f"{t1 - t0:.1f} s creation")
    small = W.bulk(L=10.0, seed=0)
    ps = oracle.make_params(**small.param_kwargs(), search=0)
    legs = {}
    for label, threads in (("bruteforce_6000_1core", 1), ("bruteforce_6000_allcores", cores)):
        oracle.set_num_threads(threads)
        o = oracle.System(ps, small.x, small.v)
        t0 = time.perf_counter()
        o.step(brute_steps)
        sec = time.perf_counter() - t0
        del o
        legs[label] = {"value": small.n * brute_steps / sec, "unit": "particle-steps/s", "cores": threads,
                       "sample": f"{brute_steps} steps of the 6,000-particle box (L = 10), O(N^2) search"}
    oracle.set_num_threads(cores)
    rate = legs["bruteforce_6000_allcores"]["value"]
    legs["bruteforce_1m_allcores_extrapolated"] = {
        "value": rate * small.n / w.n, "unit": "particle-steps/s", "cores": cores,
        "sample": "not run: the all-core O(N^2) rate of the 6,000-particle box scaled by N_small / N"}
    out["legs"] = legs
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch

    if a.copy_calibration:
        copy_calibration(a.copy_calibration)
        return

    import paper_1903_10134_amd as mdpd
    from paper_1903_10134_amd import workloads as W

    torch.cuda.set_device(0)
    if a.walled_only:
        print(json.dumps({"walled": run_walled_set(mdpd, W, a.walled)}), flush=True)
        return
    stream = torch.cuda.current_stream()
    w = W.bulk(L=a.L, seed=0)
    lanes = [int(v) for v in a.lanes.split(",")] if a.lanes else []
    res = {}
    forms = [f for f in (("fp32_forces", mdpd.FP32_FORCES, 0.0), ("fp64", mdpd.FP64, 0.0),
                         ("fp32_forces_skin", mdpd.FP32_FORCES, a.skin))
             if f[0] in a.forms.split(",")]
    for name, prec, skin in forms:
        res[name] = run_form(mdpd, w, prec, a.steps, a.warmup, a.relax, stream, lanes, skin)
        r = res[name]
        print(f"# {name}: {r['sec'] * 1e3 / a.steps:.3f} ms/step, "
              + ", ".join(f"{k} {v[0] / max(v[1], 1) * 1e3:.1f} us" for k, v in r["ktime"].items() if v[1]),
              file=sys.stderr, flush=True)

    head = res["fp32_forces"]
    n = w.n
    value = n * a.steps / head["sec"]
    full = n == 1053696 and not lanes  # the profiled configuration

    kt = head["kt_steps"]

    def kernel_roofline(kind, name, ops, alg_bytes):
        """Roofline of one kernel class on its share of the step's algorithmic
        VALU work (ops per launch), with the measured overheads as ratios."""
        ms, cnt = head["ktime"][kind]
        avg = ms / max(cnt, 1) * 1e-3
        achieved = ops / avg / 1e12
        prof = PROFILED.get(kind) if full else None
        traffic = prof["read"] + prof["write"] if prof else None
        return {"bound": "alu", "kernel": name, "achieved": achieved, "peak": PEAK_VALU_TOPS,
                "unit": "T VALU lane-ops/s", "frac": achieved / PEAK_VALU_TOPS,
                "traffic": traffic, "avg_launch_us": avg * 1e6, "launches_per_step": cnt / kt,
                "ops_per_launch": ops, "algorithmic_bytes_per_launch": alg_bytes,
                "overhead": {
                    "traffic_over_algorithmic": traffic / alg_bytes if prof else None,
                    "lane_instr_over_algorithmic": prof["valu_wave_instr"] * 64 / ops if prof else None,
                }}

    rl = {"nlist": kernel_roofline("nlist", "k_nlist_cell + k_nlist_border (FP32 form)",
                                   head["pairs_c"] * OPS_PAIR_GEOMETRY, n * BYTES_LIST),
          "density": kernel_roofline("density", "k_density (FP32 form)",
                                     head["pairs_d"] * OPS_DENSITY_PAIR, n * BYTES_DENSITY["fp32_forces"]),
          "force": kernel_roofline("force", "k_force (FP32 form)",
                                   head["pairs_c"] * OPS_PAIR_FORCE + n * OPS_VV_PARTICLE,
                                   n * BYTES_FORCE["fp32_forces"])}
    rl["nlist"]["overhead"]["candidates_per_particle"] = head["candidates"] / n
    rl["nlist"]["overhead"]["candidates_over_pairs"] = head["candidates"] / (2 * head["pairs_c"])
    dominant = max(rl, key=lambda k: rl[k]["avg_launch_us"] * rl[k]["launches_per_step"])
    out = {
        "metric": "mDPD particle-steps/s at 1M particles, FP32 vs FP64 form; adjoint/forward ratio",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": head["sec"] * 1e3 / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"bulk mDPD liquid, periodic {a.L:g}^3 box, {n} particles at density 6",
                   "n": n, "box": a.L, "A": -40.0, "B": 25.0, "rc": 1.0, "rd": 0.75, "gamma": 4.5,
                   "kT": 1.0, "dt": 0.01, "form": "FP32 pair forces + FP64 integration"},
        "forms": {},
        "roofline": rl[dominant],
        "roofline_kernels": rl,
    }
    for name, r in res.items():
        v = n * a.steps / r["sec"]
        form = "fp64" if name == "fp64" else "fp32_forces"
        bpp = BYTES_DENSITY[form] + BYTES_FORCE[form] + BYTES_RESORT * r["builds_per_step"]
        ops_step = (r["pairs_c"] * (OPS_PAIR_GEOMETRY + OPS_PAIR_FORCE) + r["pairs_d"] * OPS_DENSITY_PAIR
                    + n * OPS_VV_PARTICLE)
        out["forms"][name] = {
            "particle_steps_per_s": v,
            "ms_per_step": r["sec"] * 1e3 / a.steps,
            "kernel_us": {k: (t[0] / max(t[1], 1) * 1e3) for k, t in r["ktime"].items() if t[1]},
            "algorithmic_ops_per_particle_step": ops_step / n,
            "algorithmic_bytes_per_particle_step": bpp,
            "step_valu_frac": ops_step / (r["sec"] / a.steps) / 1e12 / PEAK_VALU_TOPS,
            "step_hbm_frac": bpp * v / 1e9 / PEAK_HBM_GBS,
            "pairs_rc": r["pairs_c"], "pairs_rd": r["pairs_d"],
            "kT_at_timing_start": r["kT_start"], "skin": r["skin"], "list_builds_per_step": r["builds_per_step"],
            "kT": r["obs"]["kT"], "pressure": r["obs"]["pressure"], "mean_rho": r["obs"]["mean_rho"],
        }
    if "fp64" in res:
        out["fp32_over_fp64"] = out["forms"]["fp32_forces"]["particle_steps_per_s"] / \
            out["forms"]["fp64"]["particle_steps_per_s"]
    if a.replicas > 0:
        bt = run_batch(mdpd, W, a.replicas, a.adj_steps, a.adj_every)
        out["batched"] = bt
        out["adjoint_over_forward"] = bt["adjoint_over_forward"]
        print(f"# batched {bt['replicas']} replicas ({bt['particles']} particles): "
              f"{bt['forward_ms_per_step']:.3f} ms/step forward ({bt['tuned_graph_forward_ms_per_step']:.3f} tuned, "
              f"graph), adjoint/forward "
              f"{bt['adjoint_over_forward']:.2f} (record+adjoint {bt['record_plus_adjoint_over_forward']:.2f})",
              file=sys.stderr, flush=True)
    if not a.no_small:
        sm = run_small(mdpd, W, 2000)
        out["small"] = sm
        print(f"# small 6000 particles: eager {sm['eager_us_per_step']:.1f} us/step, "
              f"graph {sm['graph_us_per_step']:.1f} us/step, tuned graph {sm['tuned_graph_us_per_step']:.1f} "
              f"us/step (lanes {sm['tuned_lanes']})", file=sys.stderr, flush=True)
    if not a.no_walls:
        out["walled"] = run_walled_set(mdpd, W, a.walled)
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, W, a.cpu_steps, a.brute_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
