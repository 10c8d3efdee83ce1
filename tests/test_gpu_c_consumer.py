"""The C ABI used from plain C (paper_1308_0692_amd/examples/cavity_c.c: hipMalloc'd buffers, its
own stream, no Python or PyTorch): the same solve as through the Python binding gives the same
step counts, bit-identical populations and the same centre-line velocity (the binding's results
are the ones the other GPU tests hold against the oracle)."""
import os
import subprocess

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
EXE = os.path.join(HERE, "..", "paper_1308_0692_amd", "examples", "cavity_c")


@pytest.fixture(scope="module")
def F():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1308_0692_amd as F
    return F


def test_c_consumer_equals_python_binding(F, tmp_path):
    assert os.path.exists(EXE), "examples/cavity_c is missing: run python paper_1308_0692_amd/build.py"
    n, kn, tol = 48, 0.2, 1e-9
    out = tmp_path / "f.bin"
    r = subprocess.run([EXE, str(n), str(kn), str(tol), "2", str(out)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    fields = dict(zip(r.stdout.split()[0::2], r.stdout.split()[1::2]))
    case = W.cavity(n, kn=kn, u_w=0.01, order=4)
    p = F.Problem(case, precision="mixed")
    p.init_equilibrium()
    rep = p.solve(tol, 2000000, check_every=200)
    assert int(fields["status"]) == 0 and rep["status"] == 0
    assert int(fields["steps"]) == rep["steps"] and int(fields["fp32_steps"]) == rep["steps_fp32"]
    f_c = np.fromfile(out, dtype=np.float64).reshape(p.q, n, n)
    assert np.array_equal(f_c, p.download())
    _, ux, _, _ = p.moments()
    umax = float(np.max(0.5 * (ux[:, n // 2 - 1] + ux[:, n // 2])))
    assert float(fields["centre_umax"]) == umax
