#!/usr/bin/env python3
"""Benchmark: velocity-Verlet MD of 786,432 water atoms with the DP-SE model on one GPU.

One step = one MD step of the whole hot path: displacement check against the neighbour
skin (wrap + ghost images + cell list + candidate rows rebuilt when some atom moved
more than skin/2), neighbour formatting within rc, embedding forward, descriptor +
fitting net forward and backward, embedding adjoint with force / virial scatter,
energy and virial sums (on the steps that write a thermo row, every 20), and the two
velocity-Verlet half kicks and drift.  Inputs are resident in HBM before timing.

Workload of the benchmark line: 262,144 H2O (786,432 atoms) in a 197.9 A cube, 20 steps
of 0.5 fs from 300 K (--steps), the largest configuration that fits one GPU.  Each
precision mode is timed over the same steps from the same initial state.  Its force
error is measured on the timed path itself: the forces the mode's MD returns at the
end of the timed run (Verlet list with skin, student nets with fallback) against a fresh
FP64 full-net evaluation at the same coordinates.  The students are trained on frames of
a different system (the 12,288-atom water's FP64 MD), so every frame of the timed run is
held out.  The headline value is the fastest mode whose force RMSE is at most 1e-3, as
the metric asks.  In the timed pass only the embedding adjoint (the roofline kernel) is
bracketed by HIP events; the per-stage breakdown comes from a second pass over the same
steps with every stage timed.  The FP64 CPU oracle is timed on a bounded sample (exact
forces of sampled atoms of the same frame) with all threads of the job's CPU share and
with one thread, as the CPU baseline.

Extra lines in the same JSON object ("extra"): the 12,288-atom water (100 steps of
0.5 fs, started 50 steps past the last student training frame) and FCC copper of
131,072 atoms (50 steps of 1 fs), each timed per mode the same way.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--modes ...] [--no-extras]

Modes: fp64, fp32, bf16, bf16x3 (operand precision of the embedding and fitting GEMMs),
and "<precision>+student": the student embedding nets, trained before timing on frames
of the FP64 full model's own MD (sampling, targets and fit all run in the library's
kernels), with the full net as fallback outside their s range.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "atom-steps/s on 1 GPU: FP64 vs mixed/student at force RMSE ≤1e-3 rel"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "bf16x3": 2500.0}
# vector ALU without packed FP32 instructions (the build disables them): one FMA per lane
# per cycle, 256 CUs x 4 SIMDs x 16 lanes x 2 FLOP x 2.4 GHz
ALU_PEAK_TFLOPS = 78.6
DTYPE = {"fp64": "f64", "fp32": "f32 operands, f32 accumulate", "bf16": "bf16 operands, f32 accumulate",
         "bf16x3": "bf16x3 operands, f32 accumulate"}


STUDENT_HIDDEN = 32


def algorithmic_flops(spec, rows, natoms, student=False):
    """Algorithmic FLOPs of one force evaluation (real neighbours only, no padding).
    Per neighbour row: the embedding chain (Eq. 7-9) or the student net, the
    contraction T += G^T R (Eq. 4), and in the adjoint the recomputed chain, dE/dG,
    dE/dR and the chain's input gradients.  Per atom: descriptor, fitting net forward
    and backward (Eq. 1-4)."""
    s0, s1, M = spec.emb_width
    if student:
        # the student net is affine in its hidden layer h, so the contraction and its
        # adjoint factor through per-centre products (S = sum h R^T, V = W2 dE/dT):
        # per row h (2 H + 5 H for the tanh), S += h R (8 H), and in the adjoint h again,
        # h . V (8 H), V R (8 H), dE/ds (3 H); per centre and neighbour species
        # T = W2^T S + b2 rbar^T and V, u: 8 (H + 1) M each
        H = STUDENT_HIDDEN
        emb_fwd_row = 7 * H + 8 * H + 4
        emb_bwd_row = 7 * H + 8 * H + 8 * H + 3 * H + 30
        per_centre = spec.ntypes * 8 * (H + 1) * M   # per direction, over the neighbour species
    else:
        chain = 2 * s0 + 2 * s0 * s1 + 2 * s1 * M
        chain_bwd = 2 * s1 * M + 2 * s0 * s1 + 2 * s0
        contract_row = 2 * M * 4
        emb_fwd_row = chain + contract_row
        emb_bwd_row = chain + 2 * contract_row + chain_bwd
    K1, fw, nf = spec.M * spec.m2, spec.fit_width[0], len(spec.fit_width)
    fit_atom = 2 * (2 * K1 * fw + 2 * fw * fw * (nf - 1) + 2 * fw) + 2 * spec.M * spec.m2 * 4 * 3
    # the part of the adjoint's work that is not a layer product (vector ALU): layer-0
    # affine map, tanh (counted as 5 operations: scale, exp, add, reciprocal, fma), bias
    # and skip adds, the recompute's 1 - tanh^2 factors, dE/dR = G . dE/dT (8 M), dE/ds
    # and the FP64 force / virial assembly (~30)
    if student:
        alu_bwd_row = emb_bwd_row   # all of it is vector-ALU work
        return dict(embed_fwd=rows * emb_fwd_row + natoms * per_centre,
                    embed_bwd=rows * emb_bwd_row + natoms * per_centre, fit=natoms * fit_atom,
                    emb_bwd_row=emb_bwd_row, emb_fwd_row=emb_fwd_row, fit_atom=fit_atom,
                    alu_bwd_row=alu_bwd_row, alu_bwd=rows * emb_bwd_row + natoms * per_centre,
                    per_centre=per_centre)
    else:
        ntanh = s0 + s1 + M
        alu_bwd_row = 2 * s0 + 5 * ntanh + 2 * (s1 + M) + 8 * M + 3 * ntanh + (s1 + M) + 3 * s0 + 30
    return dict(embed_fwd=rows * emb_fwd_row, embed_bwd=rows * emb_bwd_row, fit=natoms * fit_atom,
                emb_bwd_row=emb_bwd_row, emb_fwd_row=emb_fwd_row, fit_atom=fit_atom,
                alu_bwd_row=alu_bwd_row, alu_bwd=rows * alu_bwd_row)


def source_hash(files):
    """Hash of the named HIP sources (a counter-based traffic figure applies only to these)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2004_11658_amd", "csrc")
    for f in sorted(files):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def traffic_for(kernel: str):
    """HBM bytes per launch of a kernel from the committed counter summary, if it was
    measured on the current sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    k = t.get("kernels", {}).get(kernel)
    if k is None or k.get("source_hash") != source_hash(k["sources"]):
        return None
    return k["bytes_per_launch"]


POLICY = {"fp64": "NetNative<double>", "fp32": "NetNative<float>", "bf16": "NetBF16<1>", "bf16x3": "NetBF16<2>"}
STUDENT_KERNEL = {"fp64": "k_stu_bwd<double>", "fp32": "k_stu_bwd<float>", "bf16": "k_stu_bwd<float>",
                  "bf16x3": "k_stu_bwd<float>"}


def train_bench(args, path, log):
    """Training steps on a 64-frame ragged water batch (32-1024 molecules per frame):
    labels are the model's own FP64 energies and forces plus seeded noise; the timed
    region is whole steps of the training loop and, separately, the parameter gradient."""
    import numpy as np
    import torch
    from paper_2004_11658_amd import inputs as I
    from paper_2004_11658_amd import dp as D
    from paper_2004_11658_amd import train as T
    frames = I.ragged_water_batch(64, 204)
    coords = np.concatenate([f[0] for f in frames])
    types = np.concatenate([f[1] for f in frames]).astype(np.int32)
    boxes = np.stack([f[2] for f in frames])
    off = np.concatenate([[0], np.cumsum([len(f[1]) for f in frames])]).astype(np.int64)
    model = D.DPModel(path, "fp64")
    E, F, _ = model.compute_batch(coords, types, off, boxes)
    rng = np.random.default_rng(206)
    Et = E.cpu().numpy() + rng.normal(0.0, 0.5, len(frames))
    Ft = F.cpu().numpy() + rng.normal(0.0, 0.05, F.shape)
    log("training batch: %d frames, %d atoms" % (len(frames), len(types)))
    T.train(model, coords, types, off, boxes, Et, Ft, args.warmup, lr=1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    T.train(model, coords, types, off, boxes, Et, Ft, args.train_steps, lr=1e-4)
    torch.cuda.synchronize()
    dt_step = (time.perf_counter() - t0) / args.train_steps
    x = torch.as_tensor(coords, device="cuda")
    t = torch.as_tensor(types, device="cuda")
    gE = torch.ones(len(frames), dtype=torch.float64, device="cuda")
    gF = torch.full((len(types), 3), 0.1, dtype=torch.float64, device="cuda")
    model.param_grad(x, t, off, boxes, gE, gF)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.train_steps):
        model.param_grad(x, t, off, boxes, gE, gF)
    torch.cuda.synchronize()
    dt_grad = (time.perf_counter() - t0) / args.train_steps
    n = len(types)
    print(json.dumps({"metric": "training step (E + F loss, Adam)", "frames": len(frames), "atoms": n,
                      "steps": args.train_steps, "warmup": args.warmup, "ms_per_step": dt_step * 1e3,
                      "atoms_per_s": n / dt_step, "param_grad_ms": dt_grad * 1e3,
                      "param_grad_atoms_per_s": n / dt_grad, "dtype": "f64",
                      "data": "synthetic"}), flush=True)


def sig(v, d=6):
    """v to d significant digits (small values such as drifts keep their magnitude)."""
    return float("%.*g" % (d, v)) if isinstance(v, float) else v


def cpu_threads():
    """Threads of the job's CPU share: the affinity mask, capped by OMP_NUM_THREADS."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    omp = os.environ.get("OMP_NUM_THREADS")
    if omp and omp.isdigit() and int(omp) > 0:
        n = min(n, int(omp))
    return max(n, 1)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def train_student_set(D, I, S, path, masses, dt, log):
    """Students trained on frames of the FP64 full model's own MD of the 12,288-atom water
    (frames at steps 0, 10, 20, 30); also returns that trajectory's state at step 80, 50
    steps past the last training frame, where the held-out 12,288-atom run starts."""
    import torch
    full = D.DPModel(path, "fp64")
    c12, t12, b12 = I.config_water12k(202)
    v12 = I.maxwell_velocities(t12, masses, 300.0, 302)
    xs = torch.as_tensor(c12, device="cuda")
    vs = torch.as_tensor(v12, device="cuda")
    t12d = torch.as_tensor(t12, dtype=torch.int32, device="cuda")
    frames = []
    for _ in range(4):
        frames.append((xs.clone(), t12d, b12))
        full.md_run(xs, vs, t12d, masses, b12, dt, 10, 0)
    full.md_run(xs, vs, t12d, masses, b12, dt, 40, 0)
    tt = time.perf_counter()
    th, lo, hi, rep = S.train_students(full, frames, hidden=STUDENT_HIDDEN, n_samples=1_000_000)
    torch.cuda.synchronize()
    secs = time.perf_counter() - tt
    log("student training %.1f s" % secs, json.dumps(rep))
    return dict(theta=th, lo=lo, hi=hi, report=rep, seconds=secs, x12=xs, v12=vs, t12=t12d, b12=b12)


def run_modes(D, path, x0, v0, t_dev, box, masses, dt, steps, warmup, modes, skin, student, log,
              stage_pass=True):
    """Times each mode's MD from (x0, v0); its force error is that of the forces the timed
    run returns at its final coordinates against a fresh FP64 full-net evaluation there."""
    import torch
    n = x0.shape[0]
    ref = D.DPModel(path, "fp64")
    _, _, nn, _ = ref.nlist(x0, t_dev, box)
    rows = int(nn.sum().item())
    results = {}
    for mode in modes:
        prec, _, extra = mode.partition("+")
        model = D.DPModel(path, prec, skin=skin)
        if extra == "student":
            model.set_student(STUDENT_HIDDEN, student["theta"], student["lo"], student["hi"])
        x = x0.clone()
        v = v0.clone()
        model.md_run(x, v, t_dev, masses, box, dt, warmup, 0)
        x.copy_(x0)
        v.copy_(v0)
        F_end = torch.empty_like(x0)
        torch.cuda.synchronize()
        # timed pass: only the embedding adjoint (the roofline kernel) carries HIP events
        model.profile(True, stages=["embed_bwd"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        th = model.md_run(x, v, t_dev, masses, box, dt, steps, 20, forces=F_end, check=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        model.status()
        fb1 = model.fallback_rows() if extra == "student" else 0
        model.profile(False)
        bwd_timed = model.profile_read("embed_bwd")
        stages = None
        if stage_pass:
            # second pass over the same steps with every stage timed (the stage breakdown;
            # its event records slow the step, so it is not the timed pass)
            x2 = x0.clone()
            v2 = v0.clone()
            torch.cuda.synchronize()
            model.profile(True)
            model.md_run(x2, v2, t_dev, masses, box, dt, steps, 0, check=False)
            torch.cuda.synchronize()
            model.profile(False)
            stages = {s: model.profile_read(s) for s in D.STAGES}
            del x2, v2
        else:
            stages = {"embed_bwd": bwd_timed}
        stages["embed_bwd"] = bwd_timed
        del model
        # force error on the timed path: final forces vs fresh FP64 at the same coordinates
        _, Fr, _ = ref.compute(x, t_dev, box)
        dF = F_end - Fr
        rmse = float(torch.sqrt((dF * dF).mean()) / torch.sqrt((Fr * Fr).mean()))
        wall = t1 - t0
        thermo = th.cpu().numpy()
        drift = float(np.abs(thermo[:, 4] - thermo[0, 4]).max() / n)
        results[mode] = dict(value=n * steps / wall, ms_per_step=1e3 * wall / steps,
                             force_rmse_rel=rmse, energy_drift_ev_per_atom=drift,
                             temperature_K_start_end=[float(thermo[0, 3]), float(thermo[-1, 3])],
                             closest_pair_A_end=closest_pair(x, box), student=extra == "student",
                             fallback_rows_last_step=fb1,
                             stages_ms={s: v_[0] / max(v_[1], 1) for s, v_ in stages.items()},
                             stage_launches={s: v_[1] for s, v_ in stages.items()})
        log(mode, json.dumps({k: sig(v_) for k, v_ in results[mode].items() if k != "stage_launches"}))
        del x, v, F_end, Fr, dF
    del ref
    return results, rows


def closest_pair(x, box):
    """Smallest periodic distance between two atoms (A) of a cubic box, on the host.

    The synthetic potential has random weights: its tanh layers saturate as two atoms
    approach, so it holds no short-range repulsion and atoms can run into each other;
    the closest pair tells whether a run's energy drift comes from such an encounter."""
    from scipy.spatial import cKDTree
    L = float(box[0][0])
    if not np.allclose(np.asarray(box, dtype=np.float64), np.diag([L, L, L])):
        return None
    p = np.mod(x.cpu().numpy(), L)
    p[p >= L] = 0.0
    d, _ = cKDTree(p, boxsize=L).query(p, k=2)
    return float(d[:, 1].min())


def stage_rates(spec, rows, n, res):
    """Achieved TFLOP/s of the compute stages that were timed (HIP-event average per launch)."""
    fl = algorithmic_flops(spec, rows, n, student=res["student"])
    out = {}
    for st_, key in [("embed_fwd", "embed_fwd"), ("fit", "fit"), ("embed_bwd", "embed_bwd")]:
        ms = res["stages_ms"].get(st_, 0.0)
        out[st_] = sig(fl[key] / (ms * 1e-3) / 1e12) if ms > 0 else None
    return out


def summarise(results):
    def one(v_):
        if isinstance(v_, float):
            return sig(v_)
        if isinstance(v_, list):
            return [sig(u) if isinstance(u, float) else u for u in v_]
        return v_
    return {m: {k: one(v_) for k, v_ in r.items()} for m, r in results.items()}


def _counter_rows(directory):
    """Rows of every rocprofv3 counter-collection CSV under a directory."""
    import csv
    import glob
    rows = []
    for f in sorted(glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)):
        with open(f) as fh:
            rows.extend(csv.DictReader(fh))
    if not rows:
        raise SystemExit("no counter_collection.csv under %s" % directory)
    return rows


def _per_kernel(rows, counters):
    """{kernel: {counter: mean value per dispatch, "launches": n}} over the rows."""
    acc = {}
    for r in rows:
        name = r["Kernel_Name"]
        c = r["Counter_Name"]
        if c not in counters:
            continue
        k = acc.setdefault(name, {"dispatches": {}, "sum": {}})
        k["dispatches"].setdefault(c, set()).add(r["Dispatch_Id"])
        k["sum"][c] = k["sum"].get(c, 0.0) + float(r["Counter_Value"])
    out = {}
    for name, k in acc.items():
        d = {c: k["sum"][c] / len(k["dispatches"][c]) for c in k["sum"]}
        d["launches"] = max(len(v) for v in k["dispatches"].values())
        out[name] = d
    return out


def _short(name):
    """Kernel name without the namespace, argument list and launch suffix."""
    n = name.split("(")[0]
    n = n.replace("dp::", "").replace("void ", "").strip()
    return n


KERNEL_SOURCES = {"k_stu_": ["student_embed.hip", "embed_common.h", "common.h", "kernels.h"],
                  "k_fit_": ["fit_bf.hip", "common.h", "bf16ops.h", "devmath.h", "kernels.h"],
                  "k_embed_": ["embed.hip", "embed_common.h", "common.h", "bf16ops.h", "devmath.h", "kernels.h"],
                  "k_gemm": ["fit.hip", "common.h", "devmath.h", "kernels.h"],
                  "k_fb_": ["student_infer.hip", "embed_common.h", "common.h", "kernels.h"],
                  "k_nlist": ["nlist.hip", "common.h", "kernels.h"], "k_vbuild": ["nlist.hip", "common.h", "kernels.h"]}


def write_traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, workload):
    """profiles/traffic.json from four rocprofv3 runs (FETCH_SIZE and WRITE_SIZE of the
    benchmark and of a device copy of known size)."""
    cf = _per_kernel(_counter_rows(copy_fetch_dir), {"FETCH_SIZE"})
    cw = _per_kernel(_counter_rows(copy_write_dir), {"WRITE_SIZE"})
    copy_f = max(cf.items(), key=lambda kv: kv[1]["FETCH_SIZE"])[1]["FETCH_SIZE"]
    copy_w = max(cw.items(), key=lambda kv: kv[1]["WRITE_SIZE"])[1]["WRITE_SIZE"]
    copy_bytes = 256 * (1 << 20)
    fscale = copy_bytes / (copy_f * 1024.0)
    wscale = copy_bytes / (copy_w * 1024.0)
    fe = _per_kernel(_counter_rows(fetch_dir), {"FETCH_SIZE"})
    wr = _per_kernel(_counter_rows(write_dir), {"WRITE_SIZE"})
    kernels = {}
    for name in sorted(set(fe) & set(wr)):
        short = _short(name)
        srcs = next((v for k, v in KERNEL_SOURCES.items() if short.startswith(k)), None)
        if srcs is None:
            continue
        rb = fe[name]["FETCH_SIZE"] * 1024.0 * fscale
        wb = wr[name]["WRITE_SIZE"] * 1024.0 * wscale
        kernels[short] = dict(read_bytes=int(rb), written_bytes=int(wb), bytes_per_launch=int(rb + wb),
                              launches=fe[name]["launches"], sources=srcs, source_hash=source_hash(srcs))
    out = dict(note="HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE (one counter per run) on %s, "
                    "scaled by a 256 MiB device copy (read x fetch_scale, write x write_scale); an entry applies "
                    "while the hash of its source files is unchanged" % workload,
               copy_fetch_kib=copy_f, copy_write_kib=copy_w, fetch_scale=fscale, write_scale=wscale,
               kernels=kernels)
    with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: v["bytes_per_launch"] for k, v in kernels.items()}))


def mfma_table(pmc_dir):
    """Markdown table of MFMA utilisation per kernel from a rocprofv3 run that collected
    SQ_VALU_MFMA_BUSY_CYCLES, GRBM_GUI_ACTIVE and the MFMA op counters."""
    cnt = {"SQ_VALU_MFMA_BUSY_CYCLES", "GRBM_GUI_ACTIVE", "SQ_INSTS_VALU_MFMA_MOPS_BF16",
           "SQ_INSTS_VALU_MFMA_MOPS_F32", "SQ_INSTS_VALU_MFMA_MOPS_F64"}
    import csv
    import glob
    rows = _counter_rows(pmc_dir)
    dur = {}
    traces = glob.glob(os.path.join(pmc_dir, "**", "*kernel_trace.csv"), recursive=True)
    src = []
    for f in traces:
        with open(f) as fh:
            src.extend(csv.DictReader(fh))
    if not src:
        src = rows
    for r in src:
        if r.get("Start_Timestamp") and r.get("End_Timestamp"):
            dur.setdefault(r["Kernel_Name"], {})[r["Dispatch_Id"]] = float(r["End_Timestamp"]) - float(r["Start_Timestamp"])
    pk = _per_kernel(rows, cnt)
    simd = 256 * 4
    lines = ["| Kernel | Launches | MFMA busy (% of SIMD cycles) | MFMA FLOP per launch (issued) | "
             "MFMA TFLOP/s while running |", "|---|---:|---:|---:|---:|"]
    for name, d in sorted(pk.items(), key=lambda kv: -kv[1].get("SQ_VALU_MFMA_BUSY_CYCLES", 0)):
        mops = sum(d.get(c, 0.0) for c in ("SQ_INSTS_VALU_MFMA_MOPS_BF16", "SQ_INSTS_VALU_MFMA_MOPS_F32",
                                           "SQ_INSTS_VALU_MFMA_MOPS_F64"))
        if mops == 0:
            continue
        # the CSV sums GRBM_GUI_ACTIVE over the 8 XCDs (each counts the kernel's cycles)
        # and SQ_VALU_MFMA_BUSY_CYCLES over all SIMDs
        util = 100.0 * d.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) / (d.get("GRBM_GUI_ACTIVE", 1.0) / 8.0 * simd)
        ds = dur.get(name, {})
        t = sum(ds.values()) / len(ds) * 1e-9 if ds else 0.0
        rate = mops * 512 / t / 1e12 if t > 0 else float("nan")
        short = _short(name)
        if short.startswith("Cijk_"):
            short = short[:40] + "..."
        lines.append("| `%s` | %d | %.1f | %.4g | %.1f |" % (short, d["launches"], util, mops * 512, rate))
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--modes", default="fp64,fp32,bf16x3,bf16,fp32+student,bf16x3+student")
    ap.add_argument("--workload", default="water786k", choices=["water786k", "water12k"],
                    help="water786k: 786,432 atoms (the benchmark line); water12k: 12,288 atoms, started "
                         "50 steps past the last student training frame")
    ap.add_argument("--skin", type=float, default=2.0,
                    help="neighbour skin (A): the list is rebuilt when some atom moved more than skin/2")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the extra lines (12,288-atom water, 131,072-atom copper)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--train-steps", type=int, default=0,
                    help="instead of MD: time this many training steps (energies and forces, parameter "
                         "gradient of the E + F loss, Adam) on 64 ragged water frames")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="only run a device-to-device copy of this many MiB (counter calibration)")
    ap.add_argument("--calibrate-gemm", type=int, default=0,
                    help="only run torch matrix products of this size in bf16, fp32 and fp64 (MFMA counter "
                         "calibration: 2 n^3 FLOP each)")
    ap.add_argument("--write-traffic", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="only write profiles/traffic.json from rocprofv3 counter runs")
    ap.add_argument("--traffic-workload", default="the 786,432-atom water bench (bf16x3+student and fp64 modes)")
    ap.add_argument("--mfma-table", metavar="PMC_DIR", help="only print the MFMA utilisation table of a counter run")
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(*args.write_traffic, workload=args.traffic_workload)
        return
    if args.mfma_table:
        mfma_table(args.mfma_table)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the benchmark runs on one GPU only (the multi-GPU spatial decomposition is "
              "designed but not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_gemm:
        n = args.calibrate_gemm
        for dt_ in (torch.bfloat16, torch.float32, torch.float64):
            a = torch.randn(n, n, device="cuda", dtype=dt_)
            b = torch.randn(n, n, device="cuda", dtype=dt_)
            c = a @ b
            torch.cuda.synchronize()
            del a, b, c
        print(json.dumps({"gemm_n": n, "flop_each": 2 * n ** 3}))
        return
    if args.calibrate_copy_mb:
        n = args.calibrate_copy_mb * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}))
        return
    from paper_2004_11658_amd import inputs as I
    from paper_2004_11658_amd import dp as D
    from paper_2004_11658_amd import student as S

    def log(*a):
        if not args.quiet:
            print(*a, file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    spec = I.WATER
    tmp = tempfile.mkdtemp()
    path = I.write_model(os.path.join(tmp, "water.bin"), spec, I.random_params(spec, 101))
    if args.train_steps:
        train_bench(args, path, log)
        return
    masses = [I.MASS["O"], I.MASS["H"]]
    dt = 0.5
    modes = [m.strip() for m in args.modes.split(",") if m.strip()]
    if "fp64" not in modes:
        modes = ["fp64"] + modes
    student = None
    if any(m.endswith("+student") for m in modes):
        student = train_student_set(D, I, S, path, masses, dt, log)

    if args.workload == "water786k":
        coords, types, box = I.config_water786k(205)
        vel = I.maxwell_velocities(types, masses, 300.0, 305)
        x0 = torch.as_tensor(coords, device="cuda")
        v0 = torch.as_tensor(vel, device="cuda")
        t_dev = torch.as_tensor(types, dtype=torch.int32, device="cuda")
        wl = "water 786,432 atoms (262,144 H2O, 197.9 A cube)"
    else:
        assert student is not None, "the held-out 12,288-atom start comes from the student training run"
        x0, v0, t_dev, box = student["x12"].clone(), student["v12"].clone(), student["t12"], student["b12"]
        coords, types = x0.cpu().numpy(), t_dev.cpu().numpy()
        wl = "water 12,288 atoms (4,096 H2O, 49.7 A cube), 50 steps past the last student training frame"
    n = len(types)
    log("workload: %s, %d steps, dt %.2f fs" % (wl, args.steps, dt))
    results, rows = run_modes(D, path, x0, v0, t_dev, box, masses, dt, args.steps, args.warmup, modes,
                              args.skin, student, log)

    ok = [m for m in modes if results[m]["force_rmse_rel"] <= 1e-3]
    head = max(ok, key=lambda m: results[m]["value"])
    R = results[head]
    hprec = head.partition("+")[0]
    fl = algorithmic_flops(spec, rows, n, student=R["student"])
    rates = stage_rates(spec, rows, n, R)
    for m_ in modes:
        results[m_]["stage_tflops"] = stage_rates(spec, rows, n, results[m_])
    bwd_ms = R["stages_ms"]["embed_bwd"]
    achieved = fl["embed_bwd"] / (bwd_ms * 1e-3) / 1e12
    if R["student"]:
        # no matrix product per neighbour: vector-ALU bound, against the non-packed
        # FP32 / FP64 FMA rate (256 CUs x 4 SIMDs x 16 lanes x 2 FLOP x 2.4 GHz)
        kname = STUDENT_KERNEL[hprec]
        peak = ALU_PEAK_TFLOPS
        roofline = dict(bound="alu", kernel=kname, achieved=sig(achieved), peak=peak, unit="TFLOP/s",
                        frac=sig(achieved / peak, 4), traffic=traffic_for(kname),
                        flops_per_launch=fl["embed_bwd"], rows_per_launch=rows,
                        flops_per_row=fl["emb_bwd_row"], flops_per_centre=fl["per_centre"],
                        avg_launch_ms=sig(bwd_ms), stage_tflops=rates)
    else:
        peak = PEAK_TFLOPS[hprec]
        kname = "k_embed_bwd<%s, 8>" % POLICY[hprec]
        roofline = dict(bound="mfma", kernel=kname,
                        achieved=sig(achieved), peak=peak, unit="TFLOP/s",
                        frac=sig(achieved / peak, 4), traffic=traffic_for(kname),
                        flops_per_launch=fl["embed_bwd"], rows_per_launch=rows,
                        flops_per_row=fl["emb_bwd_row"], avg_launch_ms=sig(bwd_ms),
                        stage_tflops=rates,
                        alu=dict(flops_per_row=fl["alu_bwd_row"],
                                 achieved=sig(fl["alu_bwd"] / (bwd_ms * 1e-3) / 1e12),
                                 peak=ALU_PEAK_TFLOPS, unit="TFLOP/s",
                                 frac=sig(fl["alu_bwd"] / (bwd_ms * 1e-3) / 1e12 / ALU_PEAK_TFLOPS, 4)))

    extra = {}
    if not args.no_extras:
        if args.workload == "water786k" and student is not None:
            log("extra: water 12,288 atoms, 100 steps")
            r12, rows12 = run_modes(D, path, student["x12"].clone(), student["v12"].clone(), student["t12"],
                                    student["b12"], masses, dt, 100, args.warmup, modes, args.skin, student, log,
                                    stage_pass=False)
            for m_ in modes:
                r12[m_]["embed_bwd_tflops"] = stage_rates(spec, rows12, 12288, r12[m_])["embed_bwd"]
            extra["water12k"] = dict(workload="water 12,288 atoms (4,096 H2O, 49.7 A cube), 100 steps of 0.5 fs, "
                                              "started 50 steps past the last student training frame",
                                     atoms=12288, steps=100, real_neighbour_rows=rows12, modes=summarise(r12))
        log("extra: copper 131,072 atoms, 50 steps of 1 fs")
        cspec = I.COPPER
        cpath = I.write_model(os.path.join(tmp, "copper.bin"), cspec, I.random_params(cspec, 103))
        cc, ct, cb = I.config_copper131k(203)
        cm = [I.MASS["Cu"]]
        cv = I.maxwell_velocities(ct, cm, 300.0, 303)
        cmodes = [m for m in modes if not m.endswith("+student")]
        rcu, rowscu = run_modes(D, cpath, torch.as_tensor(cc, device="cuda"), torch.as_tensor(cv, device="cuda"),
                                torch.as_tensor(ct, dtype=torch.int32, device="cuda"), cb, cm, 1.0, 50,
                                args.warmup, cmodes, args.skin, None, log, stage_pass=False)
        for m_ in cmodes:
            rcu[m_]["embed_bwd_tflops"] = stage_rates(cspec, rowscu, len(ct), rcu[m_])["embed_bwd"]
        extra["copper131k"] = dict(workload="Cu FCC 32^3 cells (131,072 atoms, a 3.634 A, 0.1 A jitter), "
                                            "rc 8 A sel 512, emb 32x64x128, fit 240^3, 50 steps of 1 fs from 300 K",
                                   atoms=len(ct), steps=50, real_neighbour_rows=rowscu, modes=summarise(rcu))

    cpu = None
    if not args.no_cpu_baseline:
        from oracle.oracle import Oracle, set_threads
        nthr = cpu_threads()
        o = Oracle(path)
        rng = np.random.default_rng(7)
        runs = {}
        for thr, ns in ((nthr, 1024), (1, 64)):
            set_threads(thr)
            idx = np.sort(rng.choice(n, ns, replace=False))
            tc = time.perf_counter()
            o.eval_sampled(coords, types, box, idx)
            tc = time.perf_counter() - tc
            runs[thr] = (ns / tc, ns, tc)
        cpu = dict(value=sig(runs[nthr][0]), unit="atom-steps/s", cores=nthr, kind="oracle",
                   sample="FP64 energy and exact forces of %d sampled atoms of the first frame (the oracle's "
                          "local evaluation: every centre within rc of a sampled atom), one MD step's force "
                          "work per atom; %.1f s on %d threads" % (runs[nthr][1], runs[nthr][2], nthr),
                   single_thread=dict(value=sig(runs[1][0]), sample="%d sampled atoms, %.1f s on 1 thread"
                                      % (runs[1][1], runs[1][2])),
                   cpu_model=cpu_model(), os_cpu_count=os.cpu_count())
        log("cpu baseline", json.dumps(cpu))

    line = {
        "metric": METRIC, "value": sig(R["value"], 8), "unit": "atom-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": sig(R["ms_per_step"]),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[hprec] + (", student embedding" if R["student"] else ""), "data": "synthetic",
        "config": {"workload": wl + ", velocity-Verlet MD dt 0.5 fs from 300 K, DP-SE rc 6 A sel 46/92 emb "
                               "25x50x100 fit 240^3, random weights, neighbour skin %.1f A" % args.skin,
                   "atoms": n, "mode": head, "skin_A": args.skin, "real_neighbour_rows": rows},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "modes": summarise(results),
        "student_training": None if student is None else dict(seconds=sig(student["seconds"]),
                                                              pairs=student["report"]),
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
