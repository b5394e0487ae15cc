"""C-ABI checks that need no GPU: the library loads, exports every entry point
include/gtls.h declares, and its host helpers agree with the oracle."""
import os
import re

import numpy as np
import pytest

from paper_2607_00348_amd import gtls

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "gtls.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:gtls_status|void|int64_t|const char \*)\s*(\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    L = gtls.lib()
    names = _declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(L, name), name
    assert sorted(gtls.EXPORTED) == names


def test_params_default():
    p = gtls.gtls_params_default()
    assert (p.dt0, p.envelope, p.k_min, p.k_max, p.q_cap) == (0.0, 1, 20.05, 620.84, 0.15)
    assert (p.depth_mode, p.precision, p.median_window, p.batch_route_min) == (gtls.GTLS_DEPTH_WLS, gtls.GTLS_FP64,
                                                                               91, 3000)


def test_null_context_is_rejected():
    L = gtls.lib()
    assert L.tls_search(None, None, None, None, 0, None, 0, None, 0, None, 0, None, None) == gtls.GTLS_EINVAL
    assert L.gtls_sync(None) == gtls.GTLS_EINVAL
    L.gtls_destroy(None)


def test_create_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(gtls.GtlsError) as ei:
        gtls.Context(0)
    assert ei.value.code == gtls.GTLS_EDEVICE


@pytest.mark.parametrize("args", [(1500.0, 3.0, 1.0, 1.0, 0.0, 0.0), (89.997, 3.0, 1.0, 1.0, 0.5, 45.0),
                                  (3000.0, 3.0, 1.0, 1.0, 0.5, 1500.0), (350.0, 2.0, 0.8, 0.9, 0.0, 175.0)])
def test_period_grid_matches_oracle(oracle, args):
    a = gtls.gtls_period_grid_ofir(*args)
    b = oracle.period_grid_ofir(*args)
    assert len(a) == len(b)
    assert np.array_equal(a, b)


def test_duration_grid_matches_oracle(oracle):
    for pmin, pmax, n in ((0.5, 45.0, 12), (0.5, 1500.0, 20), (0.6018, 175.0, 20), (1.0, 2.0, 1)):
        assert np.array_equal(gtls.gtls_duration_grid(pmin, pmax, n), oracle.duration_grid(pmin, pmax, n))


@pytest.mark.parametrize("u1,u2,p,b", [(0.4, 0.25, 0.01, 0.0), (0.4, 0.25, 0.0222, 0.0), (0.3, 0.2, 0.1, 0.5),
                                       (0.4, 0.25, 0.019, 0.9), (0.0, 0.0, 0.05, 0.0)])
def test_template_matches_oracle(oracle, u1, u2, p, b):
    m = 128
    a = gtls.gtls_template_quadratic(u1, u2, p, b, m)
    ref = oracle.template_quadratic(u1, u2, p, b, m)
    assert a.max() == 1.0 and np.all(a > 0)
    assert np.max(np.abs(a - ref)) < 1e-12


def test_helpers_reject_bad_arguments():
    with pytest.raises(gtls.GtlsError):
        gtls.gtls_period_grid_ofir(-1.0)
    with pytest.raises(gtls.GtlsError):
        gtls.gtls_duration_grid(2.0, 1.0, 5)
    with pytest.raises(gtls.GtlsError):
        gtls.gtls_template_quadratic(0.4, 0.25, 0.0, 0.0, 64)


def _run_py(code: str) -> str:
    import subprocess
    import sys
    env = dict(os.environ, PYTHONPATH=ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    return out.stdout


def test_one_hip_runtime_when_library_loads_before_torch():
    """Loading the binding first and PyTorch afterwards must leave a single
    HIP runtime mapped (no GPU is touched: only the loader runs)."""
    out = _run_py("from paper_2607_00348_amd import gtls\n"
                  "gtls.lib()\n"
                  "import torch\n"
                  "print('\\n'.join(gtls._hip_runtimes()))\n")
    maps = [l for l in out.splitlines() if l.strip()]
    assert len(maps) == 1, maps


def test_two_runtimes_are_detected():
    """The failure the binding avoids: libgtls.so opened directly, before
    PyTorch, maps the ROCm install's runtime and then torch's own copy."""
    out = _run_py("import ctypes\n"
                  "from paper_2607_00348_amd import gtls\n"
                  "ctypes.CDLL(gtls.LIB_PATH)\n"
                  "import torch\n"
                  "print('\\n'.join(gtls._hip_runtimes()))\n")
    maps = [l for l in out.splitlines() if l.strip()]
    assert len(maps) == 2, maps
