"""Full-grid GPU parity on the 3000-day Kepler-like and the TESS-like
workloads at T0 step 0.1, every period against stored oracle results.

The fixtures under tests/golden/ were written by tests/golden/make_fullgrid.py,
which runs only the CPU oracle on the seeded inputs (about 15 minutes for the
3000-day curve on 8 cores).  Every period of the grid is compared:

* FP64 path: best duration, best start and the evaluation count bit-exact;
  chi2, depth and T0 to rtol 1e-9; the SDE periodogram against the oracle's
  SDE of the oracle's chi2; the best period identical.
* FP32C path: chi2 to rtol 1e-5; the best period identical; per period the
  same best window, or else a certified near-tie (never at the best period):
  the oracle's own Delta chi2 at the window the GPU chose falls short of the
  oracle's maximum by no more than the FP32C error bound of the two windows
  (storage of r, w and the template in FP32, and 32-point FP32 blocks flushed
  into FP64, give |dc| <= (2u + 32u) sum|r s| and the same for b, u = 2^-24).
"""
import os

import numpy as np
import pytest

from fp32c_bound import check_fp32c
from paper_2607_00348_amd import gtls

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
RTOL64 = 1e-9


@pytest.fixture(scope="module")
def ctx():
    c = gtls.Context(0)
    yield c
    c.close()


def _load(name):
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_fullgrid", os.path.join(HERE, "golden", "make_fullgrid.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    c, periods, durs, tm = mk.workload(name)
    fx = np.load(mk.path_of(name))
    assert str(fx["digest"]) == mk.input_digest(c, periods, durs, tm), "inputs differ from the fixture's"
    assert np.array_equal(fx["periods"], periods)
    return c, periods, durs, tm, fx


def _check_fp64(oracle, res, fx, label):
    bd, bs = fx["best_dur"].astype(np.int32), fx["best_start"]
    bad_w = np.nonzero((res.best_dur != bd) | (res.best_start != bs))[0]
    assert len(bad_w) == 0, (label, "windows differ at", bad_w[:8])
    assert np.allclose(res.chi2, fx["chi2"], rtol=RTOL64, atol=0), label
    assert np.allclose(res.depth, fx["depth"], rtol=RTOL64, atol=1e-300), label
    fin = np.isfinite(fx["t0"])
    assert np.array_equal(fin, np.isfinite(res.t0))
    assert np.allclose(res.t0[fin], fx["t0"][fin], rtol=RTOL64, atol=0), label
    assert res.n_evals == int(fx["n_evals"]), label
    assert res.chi2_null == pytest.approx(float(fx["chi2_null"]), rel=1e-15)
    sr, raw, sde, best = oracle.sde(fx["chi2"], 91)
    scale = np.max(np.abs(sde))
    assert np.allclose(res.sde, sde, rtol=0, atol=RTOL64 * scale), label
    assert np.allclose(res.sr, sr, rtol=RTOL64, atol=0), label
    assert res.best_period == best, label
    n_exact = int(np.sum(res.chi2 == fx["chi2"]))
    print(f"{label}: {len(res.chi2)} periods, windows identical, chi2 bit-identical at {n_exact}, "
          f"best period {best} (SDE {sde[best]:.2f})", flush=True)


def test_kepler_3000d_full_grid_fp64(ctx, oracle):
    c, periods, durs, tm, fx = _load("kepler_3000d")
    print("kepler_3000d full grid fp64 dt0=0.1", len(periods), flush=True)
    res = gtls.tls_search(ctx, c["t"], c["y"], c["dy"], periods, durs, tm, gtls.gtls_params_default(dt0=0.1))
    _check_fp64(oracle, res, fx, "kepler_3000d fp64")
    assert abs(periods[res.best_period] / 365.0 - 1) < 0.01


def test_kepler_3000d_full_grid_fp32c(ctx, oracle):
    c, periods, durs, tm, fx = _load("kepler_3000d")
    print("kepler_3000d full grid fp32c dt0=0.1", len(periods), flush=True)
    res = gtls.tls_search(ctx, c["t"], c["y"], c["dy"], periods, durs, tm,
                          gtls.gtls_params_default(dt0=0.1, precision=gtls.GTLS_FP32C))
    check_fp32c(oracle, c, periods, durs, tm, res, fx, "kepler_3000d fp32c")


def test_tess_full_grid_fp64(ctx, oracle):
    c, periods, durs, tm, fx = _load("tess")
    print("tess full grid fp64 dt0=0.1", len(periods), flush=True)
    res = gtls.tls_search(ctx, c["t"], c["y"], c["dy"], periods, durs, tm, gtls.gtls_params_default(dt0=0.1))
    _check_fp64(oracle, res, fx, "tess fp64")


def test_tess_full_grid_fp32c(ctx, oracle):
    c, periods, durs, tm, fx = _load("tess")
    print("tess full grid fp32c dt0=0.1", len(periods), flush=True)
    res = gtls.tls_search(ctx, c["t"], c["y"], c["dy"], periods, durs, tm,
                          gtls.gtls_params_default(dt0=0.1, precision=gtls.GTLS_FP32C))
    check_fp32c(oracle, c, periods, durs, tm, res, fx, "tess fp32c")


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
def test_proposal_label_matches_oracle(ctx, k):
    """The label of a learned-proposal training curve (the full-grid best
    period and its SDE, 418,590 periods at T0 step 0.1) as the library's search
    gives it and as the oracle gave it (tests/golden/make_fullgrid.py
    proposal_<k>).  Five curves are re-labelled: the oracle takes 30 to 45
    minutes per curve on 7 or 8 cores."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_fullgrid", os.path.join(HERE, "golden", "make_fullgrid.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    name = f"proposal_{k}"
    c, periods, durs, tm = mk.workload(name)
    fx = np.load(mk.path_of(name))
    assert str(fx["digest"]) == mk.input_digest(c, periods, durs, tm), "inputs differ from the fixture's"
    print(f"[fullgrid] {name}: n={len(c['t'])} periods={len(periods)}", flush=True)
    prm = gtls.gtls_params_default(dt0=float(fx["dt0"]))
    res = gtls.tls_search(ctx, c["t"], c["y"], c["dy"], periods, durs, tm, prm)
    assert res.best_period == int(fx["best_period"])
    assert res.sde_max == pytest.approx(float(fx["sde_max"]), rel=RTOL64)
    assert res.n_evals == int(fx["n_evals"])
