#!/usr/bin/env python3
"""MLCC2 Jacobian-transform throughput on one MI355X.

Workload: MLCC2 excitation energies on synthetic Cholesky vectors, n_occ=40,
n_vir=400, n_chol=1200, CC2 active 15 occ / 150 vir, CCS elsewhere (FP64 plain
path; the FP32 mixed path is measured beside it).

One step = one batch of n_vec=4 trial vectors (one per requested root, as in a
Davidson iteration) transformed by the full-space MLCC2 Jacobian at converged
ground-state amplitudes: X1-basis CCS terms, MLCC2 singles terms,
doubles->singles and singles->doubles (g~ derivative) contractions and the
eps_aibj doubles diagonal.  Inputs and trial vectors are resident in HBM before
the timed region.  value = transforms per second in FP64.

Also reported: FP32 transforms/s and its speedup, a full Davidson solve (4
roots to 1e-6) and a ground-state solve, the dominant contraction's achieved
TFLOP/s from HIP events on the library stream, and the FP64 oracle timed on the
host cores for one transform at the same shape.

Serving (extra.serving): a stream of MLCC2 excitation requests of uneven size
(n_occ uniform in [20, 80], n_vir = 10 n_occ, n_chol = 3 n_vir, active
0.375 n_occ / 3.75 n_occ, 3 roots, split-BF16 contractions, effective-singles
Davidson, Cholesky vectors drawn on the device) through the continuous-
batching server: first all at once (saturated solves/s), then with Poisson
arrivals at 0.7 of that rate (p50 / p99 latency from submission to a
poll-visible result).

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 157.3}
# split BF16 runs each FP32-accurate product as three dense BF16 MFMAs (2.5 PFLOP/s)
BF16_DENSE_TFLOPS = 2500.0
HBM_PEAK_GBS = 8000.0


def _cpu_baseline(timeout_s: float = 300.0):
    """Time one oracle Jacobian transform at the workload's shape on the host
    (a child process, so its BLAS threading is its own)."""
    code = r"""
import os, sys, time, json
sys.path.insert(0, %r)
import numpy as np
from oracle import mlcc as om
from paper_2006_05226_amd.synth import CONFIGS, gen_inputs, gen_amplitudes, gen_vectors
c = CONFIGS['mlcc2_40_400_1200']
inp = gen_inputs(seed=0, **c)
d = om.Dims(c['n_occ'], c['n_vir'], c['n_occ_act'], c['n_vir_act'])
P = om.Problem(inp.L, inp.eps, d, 'mlcc2')
t1, x2 = gen_amplitudes(d.O, d.V, d.o, d.v, seed=1, scale1=0.01, scale2=0.001)
c1, c2 = gen_vectors(1, d.O, d.V, d.M, seed=2)
t = time.perf_counter()
om.jacobian_transform(P, t1, x2, c1[0], c2[0].reshape(d.v, d.o, d.v, d.o))
dt = time.perf_counter() - t
try:
    cores = len(os.sched_getaffinity(0))
except Exception:
    cores = os.cpu_count()
threads = int(os.environ.get('OPENBLAS_NUM_THREADS') or os.environ.get('OMP_NUM_THREADS') or cores)
print(json.dumps(dict(seconds=dt, cores=min(cores, threads))))
""" % ROOT
    try:
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                           timeout=timeout_s)
        out = json.loads(r.stdout.strip().splitlines()[-1])
        return {"value": 1.0 / out["seconds"], "unit": "transforms/s", "cores": out["cores"],
                "kind": "oracle",
                "sample": "one complex-step FP64 Jacobian transform (1 vector) at n_occ=40, "
                          "n_vir=400, n_chol=1200, active 15/150, seeded synthetic amplitudes",
                "seconds": out["seconds"]}
    except Exception as e:  # noqa: BLE001
        return {"value": None, "unit": "transforms/s", "cores": None, "kind": "oracle",
                "sample": f"failed: {e}"}


def _profiled_traffic(tag: str, config: str, precision: str):
    """HBM bytes per launch of a contraction from its committed rocprofv3 PMC
    summary, or None when there is none or the GEMM sources changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{tag}_{config}_{precision}.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch", "kernel_source_sha256"):
            k, v = line.split(":", 1)
            fields[k] = v.strip()
    h = hashlib.sha256()
    for f in ("gemm_kernel.h", "gemm_f64.hip", "gemm_f64g.hip"):
        with open(os.path.join(ROOT, "paper_2006_05226_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if fields.get("kernel_source_sha256") != h.hexdigest() or "traffic_bytes_per_launch" not in fields:
        return None
    return float(fields["traffic_bytes_per_launch"])


def _mlccsd_leg(mlcc, steps, warmup, precisions, config="mlccsd_60_600_2000", nvec=3):
    """MLCCSD (CCS/CCSD) at its full-size workload: ground state, Jacobian
    transforms/s for a batch of nvec trial vectors, and a Davidson solve, per
    precision; Cholesky vectors drawn on the device (seed 0)."""
    import torch
    from paper_2006_05226_amd.synth import CONFIGS, gen_eps, gen_vectors

    c = CONFIGS[config]
    O, V, J, o, v = c["n_occ"], c["n_vir"], c["n_chol"], c["n_occ_act"], c["n_vir_act"]
    M = o * v
    eps = gen_eps(O, V, o, seed=0)
    c1, c2 = gen_vectors(nvec, O, V, M, seed=1)
    import numpy as np
    cvec = np.concatenate([c1.reshape(nvec, -1), c2.reshape(nvec, -1)], axis=1)
    out = {"workload": f"MLCCSD (CCS/CCSD), n_occ={O} n_vir={V} n_chol={J}, CCSD active {o}/{v}, "
                       f"device-drawn Cholesky vectors, batch of {nvec} trial vectors"}
    for prec in precisions:
        print(f"mlccsd: {prec}", file=sys.stderr, flush=True)
        ctx = mlcc.Context(0)
        P = mlcc.Problem(ctx, None, eps, O, V, o, v, model="mlccsd", precision=prec, n_chol=J,
                         seed=0)
        t0 = time.perf_counter()
        gs = P.ground_state(tol=1e-8 if prec == "fp64" else 1e-6)
        t_gs = time.perf_counter() - t0
        cd = torch.tensor(cvec, device="cuda")
        sd = torch.empty_like(cd)
        P.jacobian_transform(cd, sd)
        for _ in range(warmup):
            P.jacobian_transform(cd, sd)
        torch.cuda.synchronize()
        ctx.profile(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            P.jacobian_transform(cd, sd)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        stats = ctx.profile_stats()
        ctx.profile(False)
        t0 = time.perf_counter()
        dav = P.davidson(3, tol=1e-6)
        t_dav = time.perf_counter() - t0
        top = sorted(stats.items(), key=lambda kv: -kv[1]["ms"])[:6]
        out[prec] = dict(gs_seconds=t_gs, gs_iterations=gs["iterations"], e_corr=gs["energy"],
                         gs_converged=gs["converged"],
                         transforms_per_s=steps * nvec / dt, ms_per_step=1e3 * dt / steps,
                         davidson_seconds=t_dav, davidson_transforms=dav["transforms"],
                         omega=list(dav["omega"]), davidson_converged=dav["converged"],
                         contractions={k: dict(ms_per_step=st["ms"] / steps,
                                               tflops=st["flops"] / max(st["ms"], 1e-9) / 1e9)
                                       for k, st in top})
        P.close()
        ctx.close()
        del cd, sd
        torch.cuda.empty_cache()
    if "fp64" in out and "fp32" in out:
        out["speedup_fp32_vs_fp64"] = out["fp32"]["transforms_per_s"] / out["fp64"]["transforms_per_s"]
        out["fp32_minus_fp64"] = dict(
            e_corr=out["fp32"]["e_corr"] - out["fp64"]["e_corr"],
            omega=[a - b for a, b in zip(out["fp32"]["omega"], out["fp64"]["omega"])])
    return out


def _cnto_leg(mlcc, precisions=("fp64", "bf16x3"), config="mlcc2_40_400_1200", n_states=4):
    """Orbital selection (Sec. 2.2) at a full-size workload: CCS roots in the
    canonical basis, CNTOs from them with n_vir_act = (n_vir / n_occ) n_occ_act
    (eq. select_CNTOs), then MLCC2 on the new orbitals with their full Fock
    matrix.  Cholesky vectors drawn on the device (seed 0), canonical orbital
    energies.  The CNTO step runs twice: the first call includes the
    eigensolver library's start-up."""
    import numpy as np
    import torch
    from paper_2006_05226_amd.synth import CONFIGS, gen_eps

    c = CONFIGS[config]
    O, V, J, o = c["n_occ"], c["n_vir"], c["n_chol"], c["n_occ_act"]
    v = V * o // O
    n1, n = V * O, O + V
    eps = gen_eps(O, V, seed=0)
    # per state: gbar 4 n1^2 K, M and N 2 n1 (O^2 V + V^2 O), Z 2 V O K (V + O); then L' = C^T L C
    flops = n_states * (4.0 * n1 * n1 * J + 2.0 * n1 * (O * O * V + V * V * O)
                        + 2.0 * V * O * J * (V + O)) + 4.0 * n ** 3 * J
    out = {"workload": f"CCS roots -> CNTOs -> MLCC2, n_occ={O} n_vir={V} n_chol={J}, {n_states} "
                       f"CCS states, active {o}/{v} (n_vir_act = n_vir/n_occ x n_occ_act), "
                       f"device-drawn Cholesky vectors",
           "cnto_flops": flops}
    for prec in precisions:
        print(f"cnto: {prec}", file=sys.stderr, flush=True)
        ctx = mlcc.Context(0)
        Pc = mlcc.Problem(ctx, None, eps, O, V, 0, 0, model="ccs", precision=prec, n_chol=J, seed=0)
        t0 = time.perf_counter()
        Pc.ground_state(tol=1e-10)
        dav = Pc.davidson(n_states, tol=1e-6, want_vectors=True)
        t_ccs = time.perf_counter() - t0
        R = dav["r1"].reshape(n_states, V, O)
        R = R / np.sqrt((R * R).sum(axis=(1, 2)))[:, None, None]
        t0 = time.perf_counter()
        res = Pc.cnto(R, dav["omega"], o, v, want_L=False)
        t_cold = time.perf_counter() - t0
        ctx.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = Pc.cnto(R, dav["omega"], o, v, L_device=True)
        torch.cuda.synchronize()
        t_cnto = time.perf_counter() - t0
        stats = ctx.profile_stats()
        ctx.profile(False)
        Pc.close()
        P = mlcc.Problem(ctx, res["L"], res["eps"], O, V, o, v, model="mlcc2", precision=prec,
                         fock=res["fock"])
        res["L"] = None
        torch.cuda.empty_cache()
        t0 = time.perf_counter()
        gs = P.ground_state(tol=1e-8 if prec == "fp64" else 1e-6)
        t_gs = time.perf_counter() - t0
        t0 = time.perf_counter()
        roots = P.davidson(n_states, tol=1e-6)
        t_dav = time.perf_counter() - t0
        P.close()
        ctx.close()
        top = sorted(stats.items(), key=lambda kv: -kv[1]["ms"])[:4]
        out[prec] = dict(ccs_seconds=t_ccs, ccs_omega=list(dav["omega"]),
                         cnto_seconds=t_cnto, cnto_seconds_first_call=t_cold,
                         cnto_tflops=flops / t_cnto / 1e12,
                         m_eig_top=list(res["m_eig"][:o + 2]), n_eig_sum_active=float(np.sum(res["n_eig"][:v])),
                         n_eig_sum=float(np.sum(res["n_eig"])),
                         contractions={k: dict(ms=st["ms"], tflops=st["flops"] / max(st["ms"], 1e-9) / 1e9)
                                       for k, st in top},
                         mlcc2_gs_seconds=t_gs, mlcc2_e_corr=gs["energy"],
                         mlcc2_davidson_seconds=t_dav, mlcc2_omega=list(roots["omega"]),
                         mlcc2_converged=bool(gs["converged"] and roots["converged"]))
        del res
        torch.cuda.empty_cache()
    return out


def _c4_leg(mlcc, steps=3, nvec=5, precisions=("fp32", "bf16x3")):
    """MLCC2 at 150/1200/3600 (active 50/500), FP32 or split-BF16 contractions,
    FP64 updates, effective-singles Davidson for 5 roots; device-drawn
    Cholesky vectors.  g~ and the doubles live only in HBM (no host copies)."""
    import torch
    from paper_2006_05226_amd.synth import CONFIGS, gen_eps

    c = CONFIGS["mlcc2_150_1200_3600"]
    O, V, J, o, v = c["n_occ"], c["n_vir"], c["n_chol"], c["n_occ_act"], c["n_vir_act"]
    eps = gen_eps(O, V, o, seed=0)
    out = {"workload": f"MLCC2 n_occ={O} n_vir={V} n_chol={J}, CC2 active {o}/{v}, effective-singles "
                       "Davidson for 5 roots, device-drawn L, FP64 amplitudes/DIIS/Davidson"}
    for prec in precisions:
        print(f"c4: {prec}", file=sys.stderr, flush=True)
        ctx = mlcc.Context(0)
        t0 = time.perf_counter()
        P = mlcc.Problem(ctx, None, eps, O, V, o, v, model="mlcc2", precision=prec, n_chol=J,
                         seed=0)
        t_setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        gs = P.ground_state(tol=1e-6)
        t_gs = time.perf_counter() - t0
        c1 = torch.randn(nvec, O * V, dtype=torch.float64, device="cuda",
                         generator=torch.Generator(device="cuda").manual_seed(0)) * 1e-2
        s1 = torch.empty_like(c1)
        P.jacobian_transform_eff(0.4, c1, s1)
        torch.cuda.synchronize()
        ctx.profile(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            P.jacobian_transform_eff(0.4, c1, s1)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        stats = ctx.profile_stats()
        ctx.profile(False)
        t0 = time.perf_counter()
        dav = P.davidson(5, tol=1e-5, effective=True)
        t_dav = time.perf_counter() - t0
        peak = ctx.bytes()
        P.close()
        ctx.close()
        del c1, s1
        torch.cuda.empty_cache()
        out[prec] = {
            "setup_seconds": t_setup, "gs_seconds": t_gs, "gs_iterations": gs["iterations"],
            "e_corr": gs["energy"], "eff_transforms_per_s": steps * nvec / dt,
            "davidson_seconds": t_dav, "davidson_transforms": dav["transforms"],
            "omega": list(dav["omega"]), "davidson_converged": dav["converged"],
            "hbm_bytes_allocated": peak,
            "contractions": {k: dict(ms_per_step=st["ms"] / steps,
                                     tflops=st["flops"] / max(st["ms"], 1e-9) / 1e9)
                             for k, st in sorted(stats.items(), key=lambda kv: -kv[1]["ms"])[:8]}}
    if len(precisions) == 2:
        a, b = (out[p] for p in precisions)
        out["difference"] = dict(e_corr=b["e_corr"] - a["e_corr"],
                                 omega=[y - x for x, y in zip(a["omega"], b["omega"])])
    return out


def _serving(mlcc, n_req, slots, precision="bf16x3", rate_frac=0.7, gs_tol=1e-6, es_tol=1e-5):
    import numpy as np
    from paper_2006_05226_amd.synth import gen_eps, serving_stream

    reqs, gaps = serving_stream(n_req)
    ctx = mlcc.Context(0)
    descs = []
    for q in reqs:
        eps = gen_eps(q["n_occ"], q["n_vir"], q["n_occ_act"], q["seed"])
        descs.append(mlcc.Server.desc(None, eps, q["n_occ"], q["n_vir"], q["n_occ_act"],
                                      q["n_vir_act"], "mlcc2", precision, n_chol=q["n_chol"],
                                      seed=q["seed"]))

    def submit(srv, d):
        return srv.submit(d[0], 3, gs_tol=gs_tol, es_tol=es_tol, effective=True)

    # warm-up: one small request (first launches, allocator)
    srv = mlcc.Server(ctx, max_slots=slots)
    small = min(range(n_req), key=lambda r: reqs[r]["n_occ"])
    srv.wait(submit(srv, descs[small]))
    srv.close()

    # closed loop: every request queued at once
    srv = mlcc.Server(ctx, max_slots=slots)
    t0 = time.perf_counter()
    tickets = [submit(srv, d) for d in descs]
    burst = []
    for i, t in enumerate(tickets):
        burst.append(srv.wait(t, timeout_s=1200))
        print(f"  burst {i + 1}/{n_req} done at {time.perf_counter() - t0:.1f} s", file=sys.stderr,
              flush=True)
    wall = time.perf_counter() - t0
    srv.close()
    rate = n_req / wall
    # open loop: Poisson arrivals at rate_frac of the saturated rate
    lam = rate_frac * rate
    srv = mlcc.Server(ctx, max_slots=slots)
    t0 = time.perf_counter()
    t_next = 0.0
    tickets = []
    for d, g in zip(descs, gaps):
        t_next += g / lam
        while time.perf_counter() - t0 < t_next:
            time.sleep(min(0.002, max(0.0, t_next - (time.perf_counter() - t0))))
        tickets.append(submit(srv, d))
    stream = []
    for i, t in enumerate(tickets):
        stream.append(srv.wait(t, timeout_s=1200))
        print(f"  stream {i + 1}/{n_req} done at {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
    wall2 = time.perf_counter() - t0
    srv.close()
    ctx.close()
    lat = np.array([r["t_done"] - r["t_submit"] for r in stream])
    lat_b = np.array([r["t_done"] - r["t_submit"] for r in burst])
    ok = all(r["status"] == 0 for r in burst + stream)
    same = all(a["omega"] == b["omega"] and a["e_corr"] == b["e_corr"]
               for a, b in zip(burst, stream))
    spans = sorted((r["t_admit"], r["t_done"]) for r in stream)
    overlap = sum(1 for i in range(len(spans) - 1) if spans[i + 1][0] < spans[i][1])
    return {
        "requests": n_req, "slots": slots, "precision": precision, "roots": 3,
        "solves_per_s": rate, "burst_seconds": wall,
        "burst_latency_p50_s": float(np.percentile(lat_b, 50)),
        "arrival_rate_per_s": lam, "stream_seconds": wall2,
        "solves_per_s_stream": n_req / wall2,
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "all_ok": ok, "burst_equals_stream": same, "admissions_while_busy": overlap,
        "sizes_n_occ": [q["n_occ"] for q in reqs],
        "workload": "MLCC2 excitation requests, n_occ uniform in [20,80], n_vir=10 n_occ, "
                    f"n_chol=3 n_vir, active round(0.375 n_occ)/10x, 3 roots, {precision} contractions, "
                    "effective-singles Davidson, synthetic device-drawn Cholesky vectors",
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--nvec", type=int, default=4)
    ap.add_argument("--config", default="mlcc2_40_400_1200")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solves", action="store_true", help="skip the Davidson solve timing")
    ap.add_argument("--precisions", default="fp64,fp32,bf16x3")
    ap.add_argument("--no-mlccsd", action="store_true", help="skip the MLCCSD leg")
    ap.add_argument("--no-cnto", action="store_true", help="skip the orbital-selection leg")
    ap.add_argument("--c4", action="store_true",
                    help="also run MLCC2 at 150/1200/3600 (active 50/500), ~1 minute")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 512 MiB device copy 3 times (reference for HBM counters)")
    ap.add_argument("--serve", type=int, default=64,
                    help="requests in the serving stream (0 = skip; 256 = the full stream, "
                         "about 4 minutes)")
    ap.add_argument("--slots", type=int, default=8)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this library's hot path runs on a single MI355X; "
              "multi-GPU sharding (occupied-pair blocks, one all-reduce of the singles per "
              "transform) is designed but not built. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2006_05226_amd import mlcc
    from paper_2006_05226_amd.synth import CONFIGS, gen_inputs, gen_vectors

    if args.copy_calibration:
        src = torch.ones(1 << 26, dtype=torch.float64, device="cuda")  # 512 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    c = CONFIGS[args.config]
    O, V, J, o, v = c["n_occ"], c["n_vir"], c["n_chol"], c["n_occ_act"], c["n_vir_act"]
    M = o * v
    inp = gen_inputs(seed=0, **c)
    c1, c2 = gen_vectors(args.nvec, O, V, M, seed=1)
    cvec = np.concatenate([c1.reshape(args.nvec, -1), c2.reshape(args.nvec, -1)], axis=1)
    precs = [p for p in args.precisions.split(",") if p]
    res = {}
    for prec in precs:
        print(f"transforms: {prec}", file=sys.stderr, flush=True)
        ctx = mlcc.Context(0)
        P = mlcc.Problem(ctx, inp.L, inp.eps, O, V, o, v, model="mlcc2", precision=prec)
        t0 = time.perf_counter()
        gs = P.ground_state(tol=1e-8 if prec == "fp64" else 1e-6)
        t_gs = time.perf_counter() - t0
        cd = torch.tensor(cvec, device="cuda")
        sd = torch.empty_like(cd)
        P.jacobian_transform(cd, sd)  # builds the Jacobian intermediates
        for _ in range(args.warmup):
            P.jacobian_transform(cd, sd)
        torch.cuda.synchronize()
        ctx.profile(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            P.jacobian_transform(cd, sd)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        stats = ctx.profile_stats()
        ctx.profile(False)
        entry = dict(transforms_per_s=args.steps * args.nvec / dt, ms_per_step=1e3 * dt / args.steps,
                     gs_seconds=t_gs, gs_iterations=gs["iterations"], e_corr=gs["energy"],
                     stats=stats)
        if not args.no_solves:
            t0 = time.perf_counter()
            dav = P.davidson(4, tol=1e-6)
            entry.update(davidson_seconds=time.perf_counter() - t0,
                         davidson_transforms=dav["transforms"], omega=list(dav["omega"]),
                         davidson_converged=dav["converged"])
        res[prec] = entry
        P.close()
        ctx.close()
        del cd, sd
        torch.cuda.empty_cache()

    main_p = precs[0]
    r0 = res[main_p]
    # dominant contraction of the timed region
    st = r0["stats"]
    dom = max(st, key=lambda k: st[k]["ms"])
    d = st[dom]
    achieved = d["flops"] / (d["ms"] * 1e-3) / 1e12
    total_gemm_ms = sum(s["ms"] for s in st.values())
    traffic = _profiled_traffic(dom, args.config, main_p)
    roofline = {"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS[main_p],
                "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS[main_p], "traffic": traffic,
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                "scaled by a 512 MiB copy)",
                "kernel": dom, "launches": d["launches"],
                "avg_launch_ms": d["ms"] / d["launches"],
                "flops_per_launch": d["flops"] / d["launches"],
                "gemm_share_of_step": total_gemm_ms / (r0["ms_per_step"] * args.steps)}
    extra = {p: {k: v for k, v in e.items() if k != "stats"} for p, e in res.items()}
    for p, e in res.items():
        extra[p]["contractions"] = {k: dict(ms_per_step=s["ms"] / args.steps,
                                            tflops=s["flops"] / max(s["ms"], 1e-9) / 1e9)
                                    for k, s in sorted(e["stats"].items(),
                                                       key=lambda kv: -kv[1]["ms"])}
        # the dominant contraction of this precision against its MFMA peak(s)
        pst = e["stats"]
        pdom = max(pst, key=lambda k: pst[k]["ms"])
        pa = pst[pdom]["flops"] / (pst[pdom]["ms"] * 1e-3) / 1e12
        pr = {"kernel": pdom, "achieved_tflops": pa, "peak_tflops": PEAK_TFLOPS[p],
              "frac": pa / PEAK_TFLOPS[p]}
        if p == "bf16x3":
            pr.update(peak_note="FP32-equivalent flops; peak_tflops is the FP32 MFMA peak. "
                                "Against the BF16 matrix cores (three dense BF16 MFMAs per product):",
                      peak_bf16_three_products_tflops=BF16_DENSE_TFLOPS / 3.0,
                      frac_bf16_three_products=pa / (BF16_DENSE_TFLOPS / 3.0))
        extra[p]["roofline"] = pr
    if "fp32" in res and "fp64" in res:
        extra["speedup_fp32_vs_fp64"] = res["fp32"]["transforms_per_s"] / res["fp64"]["transforms_per_s"]
    for p in ("fp32", "bf16x3"):
        if p in res and "fp64" in res:
            extra[f"speedup_{p}_vs_fp64"] = res[p]["transforms_per_s"] / res["fp64"]["transforms_per_s"]
            if "omega" in res[p] and "omega" in res["fp64"]:
                extra[f"{p}_minus_fp64"] = dict(
                    e_corr=res[p]["e_corr"] - res["fp64"]["e_corr"],
                    omega=[a - b for a, b in zip(res[p]["omega"], res["fp64"]["omega"])])
    if args.c4:
        extra["c4"] = _c4_leg(mlcc)
    if not args.no_mlccsd:
        extra["mlccsd"] = _mlccsd_leg(mlcc, max(3, args.steps // 4), 1, precs)
    if not args.no_cnto:
        extra["cnto"] = _cnto_leg(mlcc, [p for p in ("fp64", "bf16x3") if p in precs])
    if args.serve > 0:
        print(f"serving: {args.serve} requests", file=sys.stderr, flush=True)
        extra["serving"] = _serving(mlcc, args.serve, args.slots)
    cpu = None if args.no_cpu_baseline else _cpu_baseline()
    line = {
        "metric": "Jacobian transforms/s (MLCC2, full space)",
        "value": r0["transforms_per_s"],
        "unit": "transforms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r0["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_p == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"MLCC2 Jacobian transform, n_occ={O} n_vir={V} n_chol={J}, "
                               f"CC2 active {o}/{v}, batch of {args.nvec} trial vectors",
                   "n_occ": O, "n_vir": V, "n_chol": J, "n_occ_act": o, "n_vir_act": v,
                   "n_vec": args.nvec, "precision": main_p},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
