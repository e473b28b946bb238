"""Write the oracle's dam-break observables for the long-run parity tests.

Calls only the FP64 oracle (oracle/) on the seeded synthetic inputs of
paper_2010_12375_amd.workloads; nothing here comes from the HIP path. The
observables (surge front, energies, max density deviation) are logged every
0.1 time units, as the run's observers do.

    python tests/golden/make_golden.py small      # 2D dp=0.05, seeds 0-4, t -> 1
    python tests/golden/make_golden.py medium     # 2D dp=0.00625, seed 0, t -> 20
    python tests/golden/make_golden.py medium_perturbed
        # the same run with every fluid position moved by a uniform random
        # amount of at most 2e-9 (the rounding of FP32 offsets from the cell
        # origin), to measure how far rounding alone moves the observables
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2010_12375_amd import workloads as wl  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def run(case, t_end, every=0.1, log=None):
    o = O.Oracle(case)
    o.build_config()
    rows = []
    nsub = 0
    nadv = 0
    t0 = time.time()
    k = 0
    while True:
        d = o.diagnostics()
        rows.append(dict(t=d["t"], front=d["front"], e_kin=d["e_kin"], e_pot=d["e_pot"], e_int=d["e_int"],
                         max_drho=d["max_drho"], nsub=nsub, nadv=nadv))
        if log:
            log(f"t={d['t']:.2f} front={d['front']:.5f} E={d['e_kin'] + d['e_pot'] + d['e_int']:.6f} "
                f"nsub={nsub} wall={time.time() - t0:.0f}s")
        k += 1
        T = round(every * k, 10)
        if T > t_end + 1e-12:
            break
        while o.t < T:
            nsub += o.advance(T)
            nadv += 1
    return rows, time.time() - t0


def main(which):
    if which == "small":
        out = dict(case="dambreak2d_800 (2D, dp=0.05, FP64 oracle)", t_end=1.0, seeds={})
        for seed in range(5):
            rows, wall = run(wl.config_small(seed), 1.0)
            out["seeds"][str(seed)] = rows
        path = os.path.join(HERE, "oracle_dambreak2d_800.json")
    elif which == "medium":
        case = wl.config_medium(0)
        rows, wall = run(case, 20.0, log=lambda s: print(s, flush=True))
        out = dict(case="dambreak2d_51k (2D, dp=0.00625, FP64 oracle), seed 0", t_end=20.0, seeds={"0": rows},
                   wall_seconds=wall, threads=O.num_threads())
        path = os.path.join(HERE, "oracle_dambreak2d_51k.json")
    elif which == "medium_perturbed":
        import numpy as np
        case = wl.config_medium(0)
        rng = np.random.Generator(np.random.PCG64(12345))
        case.fluid_pos = case.fluid_pos + rng.uniform(-2e-9, 2e-9, size=case.fluid_pos.shape)
        rows, wall = run(case, 20.0, log=lambda s: print(s, flush=True))
        out = dict(case="dambreak2d_51k (2D, dp=0.00625, FP64 oracle), seed 0, positions perturbed by "
                        "U(-2e-9, 2e-9), perturbation seed 12345", t_end=20.0, seeds={"0": rows},
                   wall_seconds=wall, threads=O.num_threads())
        path = os.path.join(HERE, "oracle_dambreak2d_51k_perturbed.json")
    else:
        raise SystemExit(__doc__)
    out["source"] = ("FP64 oracle (oracle/sphx_oracle.c), written by tests/golden/make_golden.py " + which)
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print("wrote", path)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "")
