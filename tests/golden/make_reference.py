"""Write oracle reference values for the full-size workloads (ground-state
correlation energy and the lowest excitation energies), for the GPU parity
tests.  Calls only the FP64 oracle and the seeded input generator.

    python tests/golden/make_reference.py mlcc2_40_400_1200 [mlccsd_60_600_2000 ...]
    python tests/golden/make_reference.py --seed 1 mlcc2_40_400_1200   # reference_<name>_seed1.json
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import mlcc as om  # noqa: E402
from paper_2006_05226_amd.synth import CONFIGS, gen_inputs  # noqa: E402

# (model, roots, ground-state tol, Davidson tol), tolerances as in the parity runs
PLAN = {
    "cc2_5_20_60": ("mlcc2", 4, 1e-11, 1e-9),
    "mlcc2_40_400_1200": ("mlcc2", 4, 1e-10, 1e-8),
    "mlccsd_60_600_2000": ("mlccsd", 3, 1e-10, 1e-8),
}


def main(names, seed=0):
    for name in names:
        model, n_roots, gs_tol, es_tol = PLAN[name]
        c = CONFIGS[name]
        t0 = time.time()
        inp = gen_inputs(seed=seed, **c)
        d = om.Dims(c["n_occ"], c["n_vir"], c["n_occ_act"], c["n_vir_act"])
        P = om.Problem(inp.L, inp.eps, d, model)
        gs = om.ground_state(P, tol=gs_tol)
        print(f"{name}: ground state E={gs['energy']:.14f} in {gs['iterations']} iterations, "
              f"{time.time() - t0:.0f} s", flush=True)
        x2 = gs.get("x2")
        dav = om.davidson(P, gs["t1"], x2, n_roots, tol=es_tol)
        out = dict(config=name, seed=seed, model=model, inputs_sha256_16=inp.digest(),
                   ground_state_tol=gs_tol, davidson_tol=es_tol,
                   e_corr=float(gs["energy"]), omega=[float(w) for w in dav["omega"]],
                   davidson_residuals=[float(r) for r in dav["residuals"]],
                   davidson_converged=bool(dav["converged"]), complex_roots=bool(dav["complex"]),
                   seconds=time.time() - t0)
        suffix = "" if seed == 0 else f"_seed{seed}"
        with open(os.path.join(HERE, f"reference_{name}{suffix}.json"), "w") as f:
            json.dump(out, f, indent=1)
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    seed = 0
    if args[:1] == ["--seed"]:
        seed, args = int(args[1]), args[2:]
    main(args or ["mlcc2_40_400_1200"], seed)
