"""Write the oracle's dam-break observables for the long-run parity tests.

Calls only the FP64 oracle (oracle/) on the seeded synthetic inputs of
paper_2010_12375_amd.workloads; nothing here comes from the HIP path. The
observables (surge front, energies, max density deviation) are logged every
0.1 time units, as the run's observers do.

    python tests/golden/make_golden.py small      # 2D dp=0.05, seeds 0-4, t -> 1
    python tests/golden/make_golden.py medium     # 2D dp=0.00625, seed 0, t -> 20
    python tests/golden/make_golden.py medium_perturbed [SEED]
        # the same run with every fluid position moved by a uniform random
        # amount of at most 2e-9 (the rounding of FP32 offsets from the cell
        # origin), to measure how far rounding alone moves the observables;
        # SEED picks the perturbation (default 12345)
    python tests/golden/make_golden.py large [T_END]
        # 3D dp=0.01 (2.0 M fluid particles), seed 0, to T_END (default 3.3,
        # past the 2 000th advection step); the file is rewritten at every
        # observer time, so an interrupted run still leaves a valid prefix
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


def run(case, t_end, every=0.1, log=None, on_row=None):
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
        if on_row:
            on_row(rows, time.time() - t0)
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


def main(which, arg=None):
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
        pseed = int(arg) if arg else 12345
        case = wl.config_medium(0)
        rng = np.random.Generator(np.random.PCG64(pseed))
        case.fluid_pos = case.fluid_pos + rng.uniform(-2e-9, 2e-9, size=case.fluid_pos.shape)
        rows, wall = run(case, 20.0, log=lambda s: print(s, flush=True))
        out = dict(case="dambreak2d_51k (2D, dp=0.00625, FP64 oracle), seed 0, positions perturbed by "
                        f"U(-2e-9, 2e-9), perturbation seed {pseed}", t_end=20.0, seeds={"0": rows},
                   wall_seconds=wall, threads=O.num_threads(), perturbation_seed=pseed)
        name = "oracle_dambreak2d_51k_perturbed.json" if pseed == 12345 else \
            f"oracle_dambreak2d_51k_perturbed_{pseed}.json"
        path = os.path.join(HERE, name)
    elif which == "large":
        t_end = float(arg) if arg else 3.3
        case = wl.config_large(0)
        path = os.path.join(HERE, "oracle_dambreak3d_2M.json")
        desc = "dambreak3d_2M (3D, dp=0.01, 2.0 M fluid + 0.596 M wall, FP64 oracle), seed 0"
        source = "FP64 oracle (oracle/sphx_oracle.c), written by tests/golden/make_golden.py large"

        def dump(rows, wall):
            part = dict(case=desc, t_end=rows[-1]["t"], t_target=t_end, seeds={"0": rows},
                        wall_seconds=wall, threads=O.num_threads(), source=source)
            with open(path + ".tmp", "w") as f:
                json.dump(part, f, indent=0)
            os.replace(path + ".tmp", path)

        rows, wall = run(case, t_end, log=lambda s: print(s, flush=True), on_row=dump)
        dump(rows, wall)
        print("wrote", path)
        return
    else:
        raise SystemExit(__doc__)
    out["source"] = ("FP64 oracle (oracle/sphx_oracle.c), written by tests/golden/make_golden.py " + which)
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print("wrote", path)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "", sys.argv[2] if len(sys.argv) > 2 else None)
