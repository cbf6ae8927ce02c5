"""Write sampled oracle states of two full-size workloads (run once; slow).

Calls only the oracle and the seeded input generators.  For each workload the
oracle runs the workload's own step count from its seeded initial state; the
file keeps the time step of every step and the conservative state at a fixed
seeded sample of cells (plus every cell of the ramp's wall row) after the
listed steps, so the GPU tests can run the same workload at full size and
compare those cells at the 1e-10 state bar.

  fullsize_ramp_1024.json   2D compression ramp 1024 x 1024, van Leer, Roe,
                            RK4, CFL 0.5: samples after 100 and 500 steps
  fullsize_box_256.json     3D jittered periodic box 256^3, van Albada, Roe,
                            RK4, CFL 0.5: samples after 50 steps

usage: python tests/golden/make_fullsize_samples.py [--resume DIR] [ramp|box ...]
(--resume DIR keeps the oracle's state there every 5 steps and continues an
interrupted run from it)
"""
import json
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

NSAMPLE = 1024


def sample_cells(case, seed):
    rng = np.random.default_rng(seed)
    cells = rng.choice(case.ncells, size=NSAMPLE, replace=False)
    return np.sort(cells)


def run(case, snapshots, cells, out_path, meta, resume_dir=None, every=5):
    """resume_dir: where to keep the oracle's state every `every` steps, so an
    interrupted run continues from its last saved step (optional)."""
    torch.set_default_dtype(torch.float64)
    P = oracle.Problem(case)
    met = P.metrics()
    Q = P.initial_state()
    dts, snaps, start = [], {}, 0
    ck = os.path.join(resume_dir, case.name + ".pt") if resume_dir else None
    if ck and os.path.exists(ck):
        saved = torch.load(ck, weights_only=True)
        Q, dts, start = list(saved["Q"]), list(saved["dt"]), int(saved["step"])
        snaps = json.loads(saved["snaps"])
        print("%s resumed at step %d" % (case.name, start), flush=True)
    idx = torch.tensor(cells, dtype=torch.long)
    t0 = time.time()
    for n in range(start + 1, max(snapshots) + 1):
        Q, dt = P.rk_step(Q, met)
        dts.append(float(dt))
        if n in snapshots:
            flat = torch.cat([q.reshape(case.nvar, -1) for q in Q], dim=1)
            snaps[str(n)] = flat[:, idx].tolist()
        print("%s step %d dt %.17g (%.0f s)" % (case.name, n, float(dt), time.time() - t0), flush=True)
        if ck and n % every == 0:
            torch.save({"Q": [q.detach() for q in Q], "dt": dts, "step": n, "snaps": json.dumps(snaps)}, ck + ".tmp")
            os.replace(ck + ".tmp", ck)
    doc = dict(meta)
    doc.update({"workload": case.name, "cells": [int(c) for c in cells], "dt": dts, "state": snaps,
                "layout": "packed conservative [var][cell], cells in k-j-i order (i fastest)",
                "written_by": "tests/golden/make_fullsize_samples.py (oracle only)"})
    with open(out_path, "w") as fh:
        json.dump(doc, fh)
    print("wrote", out_path, flush=True)


def ramp(resume_dir=None):
    case = synth.compression_ramp(1024, 1024)
    cells = np.union1d(sample_cells(case, 101), np.arange(0, 1024, 4))  # + every 4th wall-row cell
    run(case, [100, 500], cells, os.path.join(HERE, "fullsize_ramp_1024.json"),
        {"steps": 500, "generator": "synth.compression_ramp(1024, 1024)"}, resume_dir)


def box(resume_dir=None):
    case = synth.jittered_periodic_box(n=256, seed=0)
    run(case, [50], sample_cells(case, 202), os.path.join(HERE, "fullsize_box_256.json"),
        {"steps": 50, "generator": "synth.jittered_periodic_box(n=256, seed=0)"}, resume_dir)


if __name__ == "__main__":
    args = sys.argv[1:]
    resume = None
    if args[:1] == ["--resume"]:
        resume = args[1]
        os.makedirs(resume, exist_ok=True)
        args = args[2:]
    for w in args or ["ramp", "box"]:
        {"ramp": ramp, "box": box}[w](resume)
