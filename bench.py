#!/usr/bin/env python3
"""MLCC2 Jacobian-transform throughput on one MI355X.

Workload (the headline): MLCC2 excitation energies on synthetic Cholesky
vectors, n_occ=150, n_vir=1200, n_chol=3600, CC2 active 50 occ / 500 vir, CCS
elsewhere, 5 roots by the effective-singles Davidson (the doubles-doubles
block of MLCC2 is diagonal, so the doubles are eliminated at each frequency;
g~ and the eliminated doubles are built per occupied-pair block and never
stored).  Cholesky vectors drawn on the device (seed 0).

One step = one batch of n_vec=5 trial vectors (one per root) transformed by
the effective MLCC2 Jacobian A11 + A12 (w - eps)^-1 A21 at converged
ground-state amplitudes: X1-basis CCS terms, MLCC2 singles terms, the
singles -> doubles -> singles path with the FP64 denominator.  Inputs and
trial vectors are resident in HBM before the timed region.  value =
effective transforms per second with FP64 contractions; the FP32 and split-BF16
(mixed) contractions are measured beside it (extra.fp32, extra.bf16x3), with
their speedups and the energy / root differences from FP64.

Also reported: the ground state and the 5-root Davidson in each precision,
per-contraction times and TFLOP/s, the roofline of the dominant contraction
(HIP events on the library stream; HBM traffic from the committed rocprofv3
summary), the full-space MLCC2 transform at 40/400/1200 (extra.c2), MLCCSD at
60/600/2000 (extra.mlccsd), the CNTO orbital selection (extra.cnto), the
256-request serving stream (extra.serving), and the FP64 oracle on the host
cores (cpu_baseline).

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

# dense MFMA peaks of MI355X; a split-BF16 product is three dense BF16 MFMAs
# (2.5 PFLOP/s), so its FP32-equivalent peak is 2500 / 3
BF16_DENSE_TFLOPS = 2500.0
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": BF16_DENSE_TFLOPS / 3.0,
               "bf16": BF16_DENSE_TFLOPS}
PEAK_NOTE = {"fp64": "FP64 MFMA", "fp32": "FP32 MFMA",
             "bf16x3": "BF16 MFMA / 3 (each FP32-accurate product is hi*hi + hi*lo + lo*hi)",
             "bf16": "BF16 MFMA (the dominant contraction is on the plain-BF16 map: one product)"}
C4 = "mlcc2_150_1200_3600"
# the CPU-baseline sample: the same model family at a size the oracle runs in seconds
SAMPLE = dict(n_occ=30, n_vir=240, n_chol=720, n_occ_act=10, n_vir_act=100)
HBM_PEAK_GBS = 8000.0


def eff_transform_flops(n_occ, n_vir, n_chol, n_occ_act, n_vir_act):
    """Algorithmic flops of one effective MLCC2 Jacobian transformation (one
    vector): ccs_vv 2V^2OJ, ccs_W 2VO^2J, dL~ 2vo(V+O)J, the doubles block
    2M^2J twice (c2 and its contraction with L), the doubles-to-singles
    terms 2Vo vJ + 2vO oJ and jac_P 2oOVJ."""
    O, V, J, o, v = n_occ, n_vir, n_chol, n_occ_act, n_vir_act
    M = o * v
    return 2.0 * J * (V * V * O + V * O * O + v * o * (V + O) + 2.0 * M * M + V * o * v
                      + v * O * o + o * O * V)


_ORACLE_SAMPLE = r"""
import os, sys, time, json
sys.path.insert(0, %r)
import numpy as np
from oracle import mlcc as om
from paper_2006_05226_amd.synth import gen_inputs, gen_amplitudes
c = %r
inp = gen_inputs(seed=0, **c)
d = om.Dims(c['n_occ'], c['n_vir'], c['n_occ_act'], c['n_vir_act'])
P = om.Problem(inp.L, inp.eps, d, 'mlcc2')
t1, _ = gen_amplitudes(d.O, d.V, d.o, d.v, seed=1, scale1=0.01)
s = P.s_analytic(t1)
c1 = np.random.default_rng(2).standard_normal((d.V, d.O))
w = 0.4
t = time.perf_counter()
_, a21 = om.jacobian_transform(P, t1, s, c1, np.zeros((d.v, d.o, d.v, d.o)))
r1, _ = om.jacobian_transform(P, t1, s, c1, a21 / (w - om.orbital_denominators(inp.eps, d)))
dt = time.perf_counter() - t
print(json.dumps(dict(seconds=dt)))
"""


def _cpu_model():
    try:
        for line in subprocess.run(["lscpu"], capture_output=True, text=True).stdout.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:  # noqa: BLE001
        pass
    return None


def _cpu_baseline(timeout_s: float = 240.0):
    """The FP64 oracle's effective transformation (complex-step Jacobian: A21
    c1, the eliminated doubles, then A11 c1 + A12 c2) on one vector of a
    bounded sample of the workload's model family, timed in child processes
    on all host cores and pinned to one core with one BLAS thread, and scaled
    to the headline workload by the algorithmic flop ratio."""
    code = _ORACLE_SAMPLE % (ROOT, SAMPLE)
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:  # noqa: BLE001
        cores = os.cpu_count()
    ratio = eff_transform_flops(**_c4_config()) / eff_transform_flops(**SAMPLE)
    out = {"unit": "transforms/s", "kind": "oracle", "cpu_model": _cpu_model(),
           "sample": (f"one effective MLCC2 transformation (complex-step FP64 oracle) at "
                      f"n_occ={SAMPLE['n_occ']} n_vir={SAMPLE['n_vir']} n_chol={SAMPLE['n_chol']}, "
                      f"active {SAMPLE['n_occ_act']}/{SAMPLE['n_vir_act']} (the workload's "
                      f"ratios), scaled to 150/1200/3600 by the flop ratio {ratio:.0f}"),
           "flop_ratio": ratio}
    try:
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                           timeout=timeout_s)
        sec = json.loads(r.stdout.strip().splitlines()[-1])["seconds"]
        out.update(value=1.0 / (sec * ratio), cores=cores, sample_seconds=sec)
    except Exception as e:  # noqa: BLE001
        out.update(value=None, cores=None, error=f"all-core run failed: {e}")
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    try:
        r = subprocess.run(["taskset", "-c", "0", sys.executable, "-c", code], capture_output=True,
                           text=True, timeout=timeout_s, env=env)
        sec1 = json.loads(r.stdout.strip().splitlines()[-1])["seconds"]
        out.update(single_core_value=1.0 / (sec1 * ratio), single_core_sample_seconds=sec1)
    except Exception as e:  # noqa: BLE001
        out.update(single_core_value=None, single_core_error=str(e))
    return out


def _c4_config():
    from paper_2006_05226_amd.synth import CONFIGS
    return CONFIGS[C4]


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
    srcs = ("gemm_kernel.h", "gemm_f64.hip", "gemm_f64g.hip") if precision == "fp64" else \
        ("gemm_kernel.h", "gemm_split.h", "gemm_planes.h", "gemm_f32.hip", "gemm_f32d.hip",
         "gemm_f32g.hip", "gemm_f32dg.hip")
    for f in srcs:
        with open(os.path.join(ROOT, "paper_2006_05226_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if fields.get("kernel_source_sha256") != h.hexdigest() or "traffic_bytes_per_launch" not in fields:
        return None
    return float(fields["traffic_bytes_per_launch"])


def _mlccsd_leg(mlcc, steps, warmup, precisions, config="mlccsd_60_600_2000", nvec=3,
                model="mlccsd"):
    """MLCCSD (CCS/CCSD, or three-level CCS/CC2/CCSD with model "mlccsd3") at
    its full-size workload: ground state, Jacobian transforms/s for a batch of
    nvec trial vectors, and a Davidson solve, per precision; Cholesky vectors
    drawn on the device (seed 0)."""
    import torch
    from paper_2006_05226_amd.synth import CONFIGS, gen_eps, gen_vectors

    c = CONFIGS[config]
    O, V, J, o, v = c["n_occ"], c["n_vir"], c["n_chol"], c["n_occ_act"], c["n_vir_act"]
    space = (c["n_occ_ccsd"], c["n_vir_ccsd"]) if model == "mlccsd3" else None
    M = o * v
    eps = gen_eps(O, V, o, seed=0)
    c1, c2 = gen_vectors(nvec, O, V, M, seed=1)
    import numpy as np
    cvec = np.concatenate([c1.reshape(nvec, -1), c2.reshape(nvec, -1)], axis=1)
    del c1, c2
    if space:
        what = (f"three-level MLCCSD (CCS/CC2/CCSD), n_occ={O} n_vir={V} n_chol={J}, CC2 space "
                f"{o}/{v}, CCSD space {space[0]}/{space[1]}")
    else:
        what = f"MLCCSD (CCS/CCSD), n_occ={O} n_vir={V} n_chol={J}, CCSD active {o}/{v}"
    out = {"workload": f"{what}, device-drawn Cholesky vectors, batch of {nvec} trial vectors"}
    for prec in precisions:
        print(f"{model}: {prec}", file=sys.stderr, flush=True)
        ctx = mlcc.Context(0)
        P = mlcc.Problem(ctx, None, eps, O, V, o, v, model=model, precision=prec, n_chol=J,
                         seed=0, ccsd_space=space)
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
    for p in ("fp32", "bf16x3", "bf16"):
        if "fp64" in out and p in out:
            out[f"speedup_{p}_vs_fp64"] = out[p]["transforms_per_s"] / out["fp64"]["transforms_per_s"]
            out[f"{p}_minus_fp64"] = dict(
                e_corr=out[p]["e_corr"] - out["fp64"]["e_corr"],
                omega=[a - b for a, b in zip(out[p]["omega"], out["fp64"]["omega"])])
    return out


def _bf16_study(mlcc, configs=("mlcc2_40_400_1200", "mlccsd_60_600_2000"), gs_tol=1e-6, es_tol=1e-6):
    """Which contractions may run plain BF16 products (precision "bf16")?
    For each workload with FP64 oracle reference values (tests/golden), every
    contraction seen in a split-BF16 solve is run alone in plain BF16 (its
    operands rounded to BF16, one product, FP32 accumulation) and the ground
    state energy and roots are compared with the references; then all that
    pass together.  Bar: 1e-6 Eh and 1e-5 eV."""
    import numpy as np
    from paper_2006_05226_amd.synth import CONFIGS, gen_inputs
    ev = 27.211386245988
    out = {}
    for name in configs:
        with open(os.path.join(ROOT, "tests", "golden", f"reference_{name}.json")) as f:
            ref = json.load(f)
        c = CONFIGS[name]
        inp = gen_inputs(seed=0, **c)
        assert inp.digest() == ref["inputs_sha256_16"]
        ctx = mlcc.Context(0)

        def solve(tags):
            ctx.bf16_map(tags)
            P = mlcc.Problem(ctx, inp.L, inp.eps, c["n_occ"], c["n_vir"], c["n_occ_act"],
                             c["n_vir_act"], model=ref["model"], precision="bf16")
            t0 = time.perf_counter()
            g = P.ground_state(tol=gs_tol)
            d = P.davidson(len(ref["omega"]), tol=es_tol)
            sec = time.perf_counter() - t0
            P.close()
            de = abs(g["energy"] - ref["e_corr"])
            dw = float(np.abs(np.array(d["omega"]) - np.array(ref["omega"])).max())
            return dict(d_e_eh=de, d_omega_ev=dw * ev, seconds=sec,
                        ok=bool(g["converged"] and d["converged"] and de < 1e-6 and dw * ev < 1e-5))

        ctx.profile(True)
        base = solve([])
        tags = sorted(k for k in ctx.profile_stats() if k != "gemm")
        ctx.profile(False)
        rows = {"(none: split BF16 throughout)": base}
        for tag in tags:
            print(f"bf16 study {name}: {tag}", file=sys.stderr, flush=True)
            rows[tag] = solve([tag])
        passing = [t for t in tags if rows[t]["ok"]]
        rows["(all passing together)"] = solve(passing)
        out[name] = dict(rows=rows, passing=passing)
        ctx.close()
    common = sorted(set.intersection(*[set(v["passing"]) for v in out.values()]))
    out["passing_everywhere"] = common
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


def _c4_run(mlcc, prec, steps, warmup, nvec, solves, w=0.4, n_roots=5):
    """The headline workload in one precision: set-up (L drawn on the device),
    ground state, nvec effective transforms per step (the timed region), then
    the n_roots Davidson solve."""
    import numpy as np
    import torch
    from paper_2006_05226_amd.synth import gen_eps

    c = _c4_config()
    O, V, J, o, v = c["n_occ"], c["n_vir"], c["n_chol"], c["n_occ_act"], c["n_vir_act"]
    eps = gen_eps(O, V, o, seed=0)
    print(f"c4 {prec}: set-up", file=sys.stderr, flush=True)
    ctx = mlcc.Context(0)
    t0 = time.perf_counter()
    P = mlcc.Problem(ctx, None, eps, O, V, o, v, model="mlcc2", precision=prec, n_chol=J, seed=0)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    print(f"c4 {prec}: ground state", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    gs = P.ground_state(tol=1e-8 if prec == "fp64" else 1e-6)
    t_gs = time.perf_counter() - t0
    c1 = np.random.default_rng(1).standard_normal((nvec, O * V))
    c1 /= np.linalg.norm(c1, axis=1)[:, None]
    cd = torch.tensor(c1, device="cuda")
    sd = torch.empty_like(cd)
    print(f"c4 {prec}: transforms", file=sys.stderr, flush=True)
    P.jacobian_transform_eff(w, cd, sd)  # builds the Jacobian intermediates
    for _ in range(warmup):
        P.jacobian_transform_eff(w, cd, sd)
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        P.jacobian_transform_eff(w, cd, sd)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = ctx.profile_stats()
    ctx.profile(False)
    entry = dict(transforms_per_s=steps * nvec / dt, ms_per_step=1e3 * dt / steps,
                 setup_seconds=t_setup, gs_seconds=t_gs, gs_iterations=gs["iterations"],
                 e_corr=gs["energy"], gs_converged=gs["converged"], stats=stats,
                 hbm_bytes_after_transforms=ctx.bytes())
    if solves:
        print(f"c4 {prec}: davidson", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        dav = P.davidson(n_roots, tol=1e-6, effective=True)
        entry.update(davidson_seconds=time.perf_counter() - t0, davidson_transforms=dav["transforms"],
                     omega=list(dav["omega"]), davidson_converged=dav["converged"])
    entry["hbm_bytes_allocated"] = ctx.bytes()
    P.close()
    ctx.close()
    del cd, sd
    torch.cuda.empty_cache()
    return entry


def _c2_leg(mlcc, steps, warmup, precisions, nvec=4, solves=True):
    """Full-space MLCC2 Jacobian transforms/s at 40/400/1200 (active 15/150):
    batches of nvec singles+doubles trial vectors at converged amplitudes,
    host-drawn inputs (seed 0), and a 4-root full-space Davidson."""
    import numpy as np
    import torch
    from paper_2006_05226_amd.synth import CONFIGS, gen_inputs, gen_vectors

    c = CONFIGS["mlcc2_40_400_1200"]
    O, V, J, o, v = c["n_occ"], c["n_vir"], c["n_chol"], c["n_occ_act"], c["n_vir_act"]
    M = o * v
    inp = gen_inputs(seed=0, **c)
    c1, c2 = gen_vectors(nvec, O, V, M, seed=1)
    cvec = np.concatenate([c1.reshape(nvec, -1), c2.reshape(nvec, -1)], axis=1)
    out = {"workload": f"MLCC2 full-space Jacobian transform, n_occ={O} n_vir={V} n_chol={J}, "
                       f"CC2 active {o}/{v}, batch of {nvec} trial vectors"}
    for prec in precisions:
        print(f"c2: {prec}", file=sys.stderr, flush=True)
        ctx = mlcc.Context(0)
        P = mlcc.Problem(ctx, inp.L, inp.eps, O, V, o, v, model="mlcc2", precision=prec)
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
        e = dict(transforms_per_s=steps * nvec / dt, ms_per_step=1e3 * dt / steps, gs_seconds=t_gs,
                 gs_iterations=gs["iterations"], e_corr=gs["energy"],
                 contractions=_contractions(stats, steps, 8))
        if solves:
            t0 = time.perf_counter()
            dav = P.davidson(4, tol=1e-6)
            e.update(davidson_seconds=time.perf_counter() - t0, davidson_transforms=dav["transforms"],
                     omega=list(dav["omega"]), davidson_converged=dav["converged"])
        out[prec] = e
        P.close()
        ctx.close()
        del cd, sd
        torch.cuda.empty_cache()
    for p in ("fp32", "bf16x3", "bf16"):
        if p in out and "fp64" in out:
            out[f"speedup_{p}_vs_fp64"] = out[p]["transforms_per_s"] / out["fp64"]["transforms_per_s"]
    return out


def _cholesky_leg(mlcc, precisions, n_ao=160, n_aux=480, n_mo=120, n_act=40, rel_tau=1e-8):
    """Two-step Cholesky decomposition (Sec. 2.4) of synthetic AO integrals:
    the basis by pivoted Cholesky without and with the MO-screened diagonal
    (active = the first n_act MOs), then the MO Cholesky vectors by
    Algorithm 1 in each precision, with the contraction rates."""
    import numpy as np
    import torch
    from paper_2006_05226_amd.synth import gen_ao_eri, gen_mo_coefficients

    G, _ = gen_ao_eri(n_ao, n_aux, 0)
    Cmo = gen_mo_coefficients(n_ao, n_mo, 1)
    tau = rel_tau * float(np.diag(G).max())
    nu = (Cmo[:, :n_act] ** 2).max(axis=1)
    npair = n_ao * (n_ao + 1) // 2
    out = {"workload": f"AO integrals over {npair} pairs (n_ao={n_ao}, rank {n_aux}), n_mo={n_mo}, "
                       f"MO screening on {n_act} active MOs, tau = {rel_tau:g} x max diagonal"}
    ctx = mlcc.Context(0)
    Gd = torch.tensor(G, device="cuda")
    Cd = torch.tensor(Cmo, device="cuda")
    cap = n_aux + 64  # the integrals have rank n_aux
    for name, w in (("standard", None), ("mo_screened", nu)):
        print(f"cholesky basis: {name}", file=sys.stderr, flush=True)
        ctx.cholesky_basis(n_ao, Gd, tau, nu=w, max_vectors=cap)   # warm-up (library start-up)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        piv, QiT = ctx.cholesky_basis(n_ao, Gd, tau, nu=w, max_vectors=cap)
        out[f"basis_{name}"] = dict(n_vectors=len(piv), seconds=time.perf_counter() - t0)
    piv, QiT = ctx.cholesky_basis(n_ao, Gd, tau, max_vectors=cap)
    nJ = len(piv)
    flops = nJ * (2.0 * n_mo * n_ao * n_ao + 2.0 * n_mo * n_mo * n_ao) + 2.0 * nJ * nJ * n_mo * n_mo
    out["algorithm1_flops"] = flops
    for prec in precisions:
        print(f"algorithm 1: {prec}", file=sys.stderr, flush=True)
        Ld = torch.empty((nJ, n_mo, n_mo), dtype=torch.float64, device="cuda")
        ctx.mo_cholesky(n_ao, n_mo, Gd, piv, QiT, Cd, precision=prec, out=Ld)
        torch.cuda.synchronize()
        ctx.profile(True)
        t0 = time.perf_counter()
        ctx.mo_cholesky(n_ao, n_mo, Gd, piv, QiT, Cd, precision=prec, out=Ld)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = ctx.profile_stats()
        ctx.profile(False)
        out[prec] = dict(seconds=dt, tflops=flops / dt / 1e12, contractions=_contractions(st, 1))
        del Ld
    ctx.close()
    torch.cuda.empty_cache()
    return out


def _contractions(stats, steps, top=None):
    items = sorted(stats.items(), key=lambda kv: -kv[1]["ms"])
    if top:
        items = items[:top]
    return {k: dict(ms_per_step=st["ms"] / steps, launches_per_step=st["launches"] / steps,
                    tflops=st["flops"] / max(st["ms"], 1e-9) / 1e9) for k, st in items}


def _dominant_roofline(stats, prec):
    dom = max(stats, key=lambda k: stats[k]["ms"])
    d = stats[dom]
    achieved = d["flops"] / (d["ms"] * 1e-3) / 1e12
    return dom, {"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS[prec], "unit": "TFLOP/s",
                 "frac": achieved / PEAK_TFLOPS[prec], "peak_is": PEAK_NOTE[prec], "kernel": dom,
                 "launches": d["launches"], "avg_launch_ms": d["ms"] / d["launches"],
                 "flops_per_launch": d["flops"] / d["launches"]}


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
    ap.add_argument("--steps", type=int, default=4, help="timed steps (5 vectors each)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nvec", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solves", action="store_true", help="skip the Davidson solves")
    ap.add_argument("--precisions", default="fp64,fp32,bf16x3,bf16")
    ap.add_argument("--no-c2", action="store_true", help="skip the 40/400/1200 full-space leg")
    ap.add_argument("--no-mlccsd", action="store_true", help="skip the MLCCSD leg")
    ap.add_argument("--no-mlccsd3", action="store_true", help="skip the three-level MLCCSD leg")
    ap.add_argument("--no-cnto", action="store_true", help="skip the orbital-selection leg")
    ap.add_argument("--no-cholesky", action="store_true",
                    help="skip the two-step Cholesky decomposition leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 512 MiB device copy 3 times (reference for HBM counters)")
    ap.add_argument("--serve", type=int, default=256,
                    help="requests in the serving stream (0 = skip; 256 = the full stream)")
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--bf16-study", action="store_true",
                    help="only the per-contraction plain-BF16 accuracy study (prints its JSON)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this library's hot path runs on a single MI355X; "
              "multi-GPU sharding (occupied-pair blocks, one all-reduce of the singles per "
              "transform) is designed but not built. Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2006_05226_amd import mlcc

    if args.bf16_study:
        print(json.dumps(_bf16_study(mlcc)))
        return

    if args.copy_calibration:
        src = torch.ones(1 << 26, dtype=torch.float64, device="cuda")  # 512 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    c = _c4_config()
    O, V, J, o, v = c["n_occ"], c["n_vir"], c["n_chol"], c["n_occ_act"], c["n_vir_act"]
    precs = [p for p in args.precisions.split(",") if p]
    res = {p: _c4_run(mlcc, p, args.steps, args.warmup, args.nvec, not args.no_solves)
           for p in precs}
    main_p = precs[0]
    r0 = res[main_p]
    dom, roofline = _dominant_roofline(r0["stats"], main_p)
    roofline["traffic"] = _profiled_traffic(dom, C4, main_p)
    roofline["traffic_unit"] = ("HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by a "
                                "512 MiB copy)")
    total_gemm_ms = sum(st["ms"] for st in r0["stats"].values())
    roofline["gemm_share_of_step"] = total_gemm_ms / (r0["ms_per_step"] * args.steps)
    flops_vec = eff_transform_flops(O, V, J, o, v)
    extra = {"workload_flops_per_transform": flops_vec}
    for p, e in res.items():
        x = {k: val for k, val in e.items() if k != "stats"}
        x["contractions"] = _contractions(e["stats"], args.steps)
        x["sustained_tflops"] = flops_vec * e["transforms_per_s"] / 1e12
        dom_p, x["roofline"] = _dominant_roofline(e["stats"], p)
        x["roofline"]["traffic"] = _profiled_traffic(dom_p, C4, p)
        extra[p] = x
    for p in ("fp32", "bf16x3", "bf16"):
        if p in res and "fp64" in res:
            extra[f"speedup_{p}_vs_fp64"] = res[p]["transforms_per_s"] / res["fp64"]["transforms_per_s"]
            d = dict(e_corr_eh=res[p]["e_corr"] - res["fp64"]["e_corr"])
            if "omega" in res[p] and "omega" in res["fp64"]:
                d["omega_eh"] = [a - b for a, b in zip(res[p]["omega"], res["fp64"]["omega"])]
                d["omega_ev"] = [x * 27.211386245988 for x in d["omega_eh"]]
            extra[f"{p}_minus_fp64"] = d
    if not args.no_c2:
        extra["c2"] = _c2_leg(mlcc, max(5, 5 * args.steps), 2, precs, solves=not args.no_solves)
    if not args.no_mlccsd:
        extra["mlccsd"] = _mlccsd_leg(mlcc, max(3, args.steps), 1, precs)
    if not args.no_mlccsd3:
        extra["mlccsd3"] = _mlccsd_leg(mlcc, max(3, args.steps), 1, precs,
                                       config="mlccsd3_60_600_2000", model="mlccsd3")
    if not args.no_cnto:
        extra["cnto"] = _cnto_leg(mlcc, [p for p in ("fp64", "bf16x3") if p in precs])
    if not args.no_cholesky:
        extra["cholesky"] = _cholesky_leg(mlcc, precs)
    if args.serve > 0:
        print(f"serving: {args.serve} requests", file=sys.stderr, flush=True)
        extra["serving"] = _serving(mlcc, args.serve, args.slots)
    cpu = None if args.no_cpu_baseline else _cpu_baseline()
    line = {
        "metric": "Jacobian transforms/s (MLCC2, effective singles)",
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
        "config": {"workload": f"MLCC2 effective-singles Jacobian transform, n_occ={O} n_vir={V} "
                               f"n_chol={J}, CC2 active {o}/{v}, batch of {args.nvec} trial vectors, "
                               "device-drawn Cholesky vectors",
                   "n_occ": O, "n_vir": V, "n_chol": J, "n_occ_act": o, "n_vir_act": v,
                   "n_vec": args.nvec, "precision": main_p},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
