"""The precision form: volumes, projections and CGLS vectors stored in FP16
or BF16 (FP32 arithmetic, FP64 reductions), against the FP64 oracle.

The error of each result is reported (printed); the bounds asserted here are
loose guards against breakage, not accuracy claims: FP16 keeps 11
significant bits (relative spacing 9.8e-4), BF16 8 bits (7.8e-3).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1008_2042_amd import inputs, metrics

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1008_2042_amd import tfcb  # noqa: E402

DT = {"f16": (tfcb.F16, 2e-3, 3e-2), "bf16": (tfcb.BF16, 1.5e-2, 8e-2)}


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


@pytest.mark.parametrize("name", ["f16", "bf16"])
def test_operators_in_storage_dtype(name):
    dev = _dev()
    code, op_tol, _ = DT[name]
    tdt = tfcb.torch_dtype(code)
    g = inputs.config("tiny")["geom"]
    f = inputs.random_volume(g, 21)
    y = inputs.random_sino(g, 22)
    print("[gpu-case] operators %s" % name, flush=True)
    pf = tfcb.project(g, torch.tensor(f, device=dev).to(tdt))
    pty = tfcb.backproject(g, torch.tensor(y, device=dev).to(tdt))
    torch.cuda.synchronize()
    e1 = rel(pf.float().cpu().numpy(), oracle.project(g, f))
    e2 = rel(pty.float().cpu().numpy(), oracle.backproject(g, y))
    print("%s: P rel L2 %.2e, P^T rel L2 %.2e" % (name, e1, e2))
    assert e1 <= op_tol and e2 <= op_tol


@pytest.mark.parametrize("cfg_name", ["precision", "precision_5e4"])
def test_precision_form_reconstruction(cfg_name):
    dev = _dev()
    cfg = inputs.config(cfg_name)
    g = cfg["geom"]
    y = inputs.measured_data(cfg)
    ref, _ = oracle.reconstruct(g, y, cfg["lam"], cfg["iters"])
    ells = inputs.phantom_for(cfg)
    cnr_ref = np.array(metrics.cnr_all(ref, g, ells))
    yd = torch.tensor(y, dtype=torch.float32, device=dev)
    rows = []
    for name, code in (("f32", tfcb.F32), ("f16", tfcb.F16), ("bf16", tfcb.BF16)):
        print("[gpu-case] reconstruct %s %s" % (cfg_name, name), flush=True)
        got, rep = tfcb.reconstruct(g, yd, cfg["lam"], cfg["iters"], storage=code)
        v = got.cpu().numpy().astype(np.float64)
        assert np.all(np.isfinite(v))
        e = rel(v, ref)
        cnr = np.array(metrics.cnr_all(v, g, ells))
        cnr_err = float(np.max(np.abs(cnr - cnr_ref) / np.abs(cnr_ref)))
        rows.append((name, e, cnr_err))
        print("%s %s: rel L2 vs FP64 oracle %.3e, max relative CNR error %.3e"
              % (cfg_name, name, e, cnr_err))
        sys.stdout.flush()
        bound = 1e-3 if name == "f32" else DT[name][2]
        assert e <= bound, (name, e)
