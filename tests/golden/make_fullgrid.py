"""Write the full-grid oracle fixtures of the 3000-day and TESS-like workloads.

Calls only the CPU oracle (``oracle/``) and the seeded input generators
(``paper_2607_00348_amd/synth.py``, which hold no search arithmetic).  Each
fixture stores, for every period of the workload's Ofir grid, the oracle's
chi2, best duration index, best window start, depth and T0 at the T0 step
dt0 = 0.1 (Sect. 2.5), plus the grid itself and a description of the inputs.
The GPU tests compare every period of the library's search with these arrays.
For five curves of the learned-proposal set (3000-day curves, the same
418,590-period grid) it stores only the label, the full-grid best period and
its SDE, with the evaluation count and a digest of the oracle's chi2 array.

    python tests/golden/make_fullgrid.py [kepler_3000d|tess|proposal_<k>] [--threads N]

Run time: about 15 minutes for the 3000-day curve on 8 cores, about 2 for the
TESS-like curve, 30 to 45 for each proposal curve on 7 or 8.
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2607_00348_amd import synth  # noqa: E402

DT0 = 0.1


PROPOSAL_CURVES = (0, 1, 2, 3, 4)


def proposal_grid():
    """Grid of the learned-proposal set: the 3000-day cadence grid's span,
    Ofir periods 0.5-1500 d at oversampling 3, 20 durations."""
    span = (int(round(3000.0 / synth.KEPLER_CADENCE_DAYS)) - 1) * synth.KEPLER_CADENCE_DAYS
    periods = O.period_grid_ofir(span, 3.0, pmin_days=0.5, pmax_days=1500.0)
    durs = O.duration_grid(0.5, 1500.0, 20)
    return periods, durs


def workload(name: str):
    """Inputs and grids of one workload, exactly as the GPU tests build them."""
    if name.startswith("proposal_"):
        c = synth.proposal_curve(int(name.split("_")[1]))
        periods, durs = proposal_grid()
    elif name == "kepler_3000d":
        c = synth.curve_3000d()
        span = c["t"][-1] - c["t"][0]
        periods = O.period_grid_ofir(span, 3.0, pmin_days=0.5, pmax_days=1500.0)
        durs = O.duration_grid(0.5, 1500.0, 20)
    elif name == "tess":
        c = synth.curve_tess()
        span = c["t"][-1] - c["t"][0]
        periods = O.period_grid_ofir(span, 3.0, pmax_days=175.0)
        durs = O.duration_grid(periods[0], periods[-1], 20)
    else:
        raise ValueError(name)
    tm = O.template_quadratic(0.4, 0.25, 0.01, 0.0, 1024)
    return c, periods, durs, tm


def input_digest(c, periods, durs, tm) -> str:
    h = hashlib.sha256()
    for a in (c["t"], c["y"], c["dy"], periods, durs, tm):
        h.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    return h.hexdigest()


def path_of(name: str) -> str:
    return os.path.join(HERE, f"fullgrid_{name}_dt0_0.1.npz")


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*", default=["tess", "kepler_3000d"] + [f"proposal_{k}" for k in PROPOSAL_CURVES])
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    for name in a.names:
        c, periods, durs, tm = workload(name)
        print(f"{name}: n={len(c['t'])} periods={len(periods)} durations={len(durs)}", flush=True)
        t0 = time.time()
        ref = O.tls_search(c["t"], c["y"], c["dy"], periods, durs, tm, dt0=DT0, threads=a.threads)
        el = time.time() - t0
        print(f"{name}: oracle {el:.1f} s, {ref.n_evals} evaluations", flush=True)
        if name.startswith("proposal_"):
            # labels of the learned proposal: the best period of the full-grid
            # periodogram (largest SDE), its SDE, and a digest of the chi2 array
            _, _, sde, best = O.sde(ref.chi2, 91)
            np.savez_compressed(path_of(name), best_period=np.int64(best), sde_max=np.float64(sde[best]),
                                chi2_sha256=np.array(hashlib.sha256(ref.chi2.tobytes()).hexdigest()),
                                n_evals=np.int64(ref.n_evals), digest=np.array(input_digest(c, periods, durs, tm)),
                                dt0=np.float64(DT0))
            continue
        np.savez_compressed(path_of(name), periods=periods, chi2=ref.chi2,
                            best_dur=ref.best_dur.astype(np.int8), best_start=ref.best_start,
                            depth=ref.depth, t0=ref.t0, chi2_null=np.float64(ref.chi2_null),
                            n_evals=np.int64(ref.n_evals), digest=np.array(input_digest(c, periods, durs, tm)),
                            dt0=np.float64(DT0))


if __name__ == "__main__":
    main()
