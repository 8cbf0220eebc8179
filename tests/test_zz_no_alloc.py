"""The backprojector entry point that allocates nothing
(tfcb_backproject_noalloc) against tfcb_backproject, which carves the same
scratch from a caller workspace: same kernels, so the results must agree bit
for bit.  Two calls in a row share the static scratch array, the second on a
smaller geometry; a geometry whose scratch need exceeds the array is refused
before anything is enqueued."""
from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1008_2042_amd import inputs, tfcb  # noqa: E402

pytestmark = pytest.mark.gpu

# about 11.8 MB of prescaled FP32 projections, then a 0.98 MB one
LARGER = inputs.Geometry(256, 256, 48, 1.0, 1.0, 3.6, 256, 192, 1.55, 1.55, n_views=60)
SMALLER = inputs.Geometry(64, 64, 16, 1.0, 1.0, 1.0, 128, 64, 1.5, 1.5, n_views=30)


def _need():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    tfcb.load()
    return torch.device("cuda:0")


@pytest.mark.parametrize("dtype", [torch.float32, torch.float16], ids=["f32", "f16"])
def test_noalloc_matches_workspace_entry_point(dtype):
    dev = _need()
    for g, seed in ((LARGER, 11), (SMALLER, 12)):
        print("noalloc backprojection: %dx%dx%d, %d views of %dx%d, %s"
              % (g.nx, g.ny, g.nz, g.n_views, g.nu, g.nv, dtype), flush=True)
        proj = torch.tensor(inputs.random_sino(g, seed), dtype=dtype, device=dev)
        want = tfcb.backproject(g, proj)
        got = torch.full_like(want, float("nan"))
        tfcb.backproject_noalloc(g, proj, out=got)
        torch.cuda.synchronize()
        assert torch.isfinite(got).all()
        assert torch.equal(got, want), float((got.float() - want.float()).abs().max())


def test_noalloc_smaller_call_against_oracle():
    import oracle
    dev = _need()
    g = SMALLER
    y = inputs.random_sino(g, 13)
    got = tfcb.backproject_noalloc(g, torch.tensor(y, dtype=torch.float32, device=dev))
    torch.cuda.synchronize()
    want = oracle.backproject(g, y)
    rel = float(np.linalg.norm(got.cpu().numpy() - want) / np.linalg.norm(want))
    print("noalloc P^T vs FP64 oracle: relative L2 %.2e" % rel, flush=True)
    assert rel <= 1e-4


def test_noalloc_refuses_oversize_geometry():
    dev = _need()
    big = inputs.config("large")["geom"]  # 360 x 768 x 1024 projections: 1.13 GB of scratch
    dummy = torch.zeros(16, dtype=torch.float32, device=dev)
    out = torch.zeros(16, dtype=torch.float32, device=dev)
    with pytest.raises(tfcb.TfcbError) as e:
        tfcb.load()
        tfcb._check(tfcb.load().tfcb_backproject_noalloc(
            tfcb.ctypes.byref(tfcb.geometry(big)), tfcb.F32, tfcb._ptr(dummy), tfcb._ptr(out),
            tfcb._stream(None)))
    assert e.value.status == tfcb.EUNSUPPORTED
    assert "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((out == 0).all())
