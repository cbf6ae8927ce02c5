"""Full-size multi-step parity against stored oracle samples.

tests/golden/make_fullsize_samples.py (which calls only the oracle) ran the
full workloads from their seeded initial states and stored every step's time
step and the conservative state at a seeded sample of cells (plus part of the
ramp's wall row).  Here the HIP path runs the same workloads at full size, in
the launch configuration the bench times, and is compared on those cells at
the state bar (1e-10 of the free-stream scale per variable) and on every time
step at 1e-12 relative."""
import json
import os
import sys

import pytest
import torch

import synth
from parity_util import STATE_TOL, q_ref

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _load(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip("%s not generated (tests/golden/make_fullsize_samples.py)" % name)
    with open(path) as fh:
        return json.load(fh)


def _run_and_compare(case, doc, variant=None, mode=None):
    from paper_2012_02925_amd.solver import Solver
    s = Solver.from_case(case, device="cuda:0")
    if variant is not None:
        s.set_variant(variant)
    if mode is not None:
        s.set_exec(mode, True)
    cells = torch.tensor(doc["cells"], dtype=torch.long)
    qr = torch.tensor(q_ref(case), dtype=torch.float64)
    dt = torch.empty(1, dtype=torch.float64, device="cuda:0")
    nsteps = doc["steps"]
    worst_dt = 0.0
    for n in range(1, nsteps + 1):
        s.rk_step(1, dt)
        ref = doc["dt"][n - 1]
        worst_dt = max(worst_dt, abs(dt.item() - ref) / ref)
        if str(n) in doc["state"]:
            Q = s.get_state()[:, cells.to("cuda:0")].cpu()
            Qref = torch.tensor(doc["state"][str(n)], dtype=torch.float64)
            err = ((Q - Qref).abs().amax(dim=1) / qr)
            _say("  step %d: max state error / Q_ref per variable %s" % (n, err.tolist()))
            assert bool(torch.isfinite(Q).all())
            assert bool((err <= STATE_TOL).all()), (n, err.tolist())
    _say("  worst dt relative error %.3e" % worst_dt)
    assert worst_dt <= 1e-12
    s.close()


@pytest.mark.parametrize("variant", [None, 0])
def test_ramp_1024_500_steps(variant):
    """Config of the 2D compression ramp: 1024^2 cells, van Leer, Roe, RK4,
    CFL 0.5, 500 steps from the uniform free stream; samples after 100 and
    500 steps (autotuned-default and a second tile variant)."""
    doc = _load("fullsize_ramp_1024.json")
    _say("case: compression ramp 1024^2, 500 steps, variant", variant)
    _run_and_compare(synth.compression_ramp(1024, 1024), doc, variant)


@pytest.mark.parametrize("mode", ["batched", "persistent"])
def test_box_256_50_steps(mode):
    """The headline workload: 256^3 jittered periodic box, van Albada, Roe,
    RK4, CFL 0.5, 50 steps; samples after 50 steps."""
    doc = _load("fullsize_box_256.json")
    _say("case: jittered periodic box 256^3, 50 steps,", mode)
    _run_and_compare(synth.jittered_periodic_box(n=256, seed=0), doc, mode=mode)
