"""The large single-reconstruction workload (512x512x256 at 0.5 mm, 360 views
of a 1024x768 detector at 0.388 mm) at its real shape: sampled projector
outputs against the oracle, the adjoint identity of the full-size operators,
sampled framelet outputs at one and two levels, and a shortened 3-grid,
2-level-framelet reconstruction."""
import sys

import numpy as np
import pytest

import oracle
from paper_1008_2042_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1008_2042_amd import tfcb  # noqa: E402

LARGE = inputs.config("large")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def announce(msg):
    print("[gpu-case]", msg, flush=True)
    sys.stdout.flush()


def test_large_project_sampled_and_adjoint():
    dev = _dev()
    g = LARGE["geom"]
    f = inputs.random_volume(g, 41)
    announce("large project")
    fd = torch.tensor(f, dtype=torch.float32, device=dev)
    pf = tfcb.project(g, fd)
    rng = np.random.default_rng(42)
    vrc = np.stack([rng.integers(0, g.n_views, 128), rng.integers(0, g.nv, 128),
                    rng.integers(0, g.nu, 128)], axis=1)
    got = pf[vrc[:, 0], vrc[:, 1], vrc[:, 2]].double().cpu().numpy()
    want = oracle.project_rays(g, f, vrc)
    assert np.linalg.norm(got - want) / np.linalg.norm(want) <= 1e-4
    announce("large adjoint identity")
    gen = torch.Generator(device=dev)
    gen.manual_seed(43)
    y = torch.rand(g.sino_shape, generator=gen, device=dev, dtype=torch.float32) * 2 - 1
    pty = tfcb.backproject(g, y)
    lhs = float(torch.sum(pf.double() * y.double()))
    rhs = float(torch.sum(fd.double() * pty.double()))
    scale = float(torch.linalg.norm(pf.double()) * torch.linalg.norm(y.double()))
    err = abs(lhs - rhs) / scale
    print("large adjoint identity: mismatch %.2e of ||Pf|| ||y||, %.2e of <Pf, y>"
          % (err, abs(lhs - rhs) / abs(lhs)), flush=True)
    assert err <= 1e-7


@pytest.mark.parametrize("levels", [1, 2])
def test_large_framelet_sampled(levels):
    """The fused framelet shrink at 512x512x256 (several z chunks per column
    of blocks, and with two levels the dilation-2 chains of both z residues)
    at sampled voxels, faces and corners included, against the oracle."""
    dev = _dev()
    g = LARGE["geom"]
    f = inputs.random_volume(g, 44)
    lam = 2e-3
    announce("large framelet levels=%d" % levels)
    got = tfcb.framelet_shrink(torch.tensor(f, dtype=torch.float32, device=dev), lam, levels,
                               True).double().cpu().numpy()
    rng = np.random.default_rng(45)
    kji = np.stack([rng.integers(0, g.nz, 48), rng.integers(0, g.ny, 48),
                    rng.integers(0, g.nx, 48)], axis=1)
    edges = np.array([[0, 0, 0], [g.nz - 1, g.ny - 1, g.nx - 1], [0, g.ny // 2, g.nx - 1],
                      [g.nz - 1, 0, g.nx // 3], [1, 1, 1], [g.nz - 2, g.ny - 2, 5],
                      [g.nz // 2, 0, 0], [g.nz // 2 + 1, g.ny - 1, g.nx - 2]])
    kji = np.concatenate([kji, edges])
    want = oracle.framelet_shrink_voxels(f, lam, kji, levels, True)
    a = got[kji[:, 0], kji[:, 1], kji[:, 2]]
    assert np.linalg.norm(a - want) <= 1e-5 * np.linalg.norm(want)


@pytest.mark.parametrize("storage", [tfcb.F32, tfcb.F16])
def test_large_reconstruction_shortened(storage):
    """Three grids and two framelet levels, one iteration per grid."""
    dev = _dev()
    g = LARGE["geom"]
    announce("large reconstruct storage=%d" % storage)
    ells = inputs.phantom_for(LARGE)
    y = inputs.analytic_projection_torch(g, ells, dev).float()
    vol, rep = tfcb.reconstruct(g, y, LARGE["lam"], [1, 1, 1], framelet_levels=2,
                                storage=storage)
    v = vol.cpu().numpy()
    assert np.all(np.isfinite(v)) and v.min() >= 0.0
    assert rep["iters_done"] == [1, 1, 1]
    assert rep["resid2_last"] < 0.5 * float(torch.sum(y.double() ** 2))


@pytest.mark.timeout(900)
def test_large_coarsest_grid_iteration_whole_volume():
    """One full outer iteration of Algorithm A2 (3 CGLS steps, two-level
    framelet shrink, positivity) on the coarsest grid of the large workload's
    3-grid schedule (128x128x64 at 2 mm, 360 views of the twice-binned
    256x192 detector at 1.552 mm), from zero, over the whole volume against
    the FP64 oracle: FP32 within 1e-3, FP16 storage reported (guard 1e-2).
    The data are exact chords through the workload's 40-ellipsoid phantom
    with Poisson noise (I0 = 5e4), generated on that geometry."""
    dev = _dev()
    gf = LARGE["geom"]
    g = inputs.Geometry(gf.nx // 4, gf.ny // 4, gf.nz // 4, 4 * gf.dx, 4 * gf.dy, 4 * gf.dz,
                        gf.nu // 4, gf.nv // 4, 4 * gf.du, 4 * gf.dv, sad=gf.sad, sdd=gf.sdd,
                        n_views=gf.n_views)
    announce("large coarsest-grid data %dx%dx%d, %d views of %dx%d"
             % (g.nx, g.ny, g.nz, g.n_views, g.nu, g.nv))
    clean = inputs.analytic_projection_torch(g, inputs.phantom_for(LARGE), dev)
    y = inputs.poisson_log_torch(clean, LARGE["noise"][0], LARGE["noise"][1]).cpu().numpy()
    del clean
    announce("FP64 oracle: one outer iteration on %d threads" % oracle.num_threads())
    want, orep = oracle.reconstruct(g, y, LARGE["lam"], [1], LARGE["cgls_steps"],
                                    LARGE["framelet_levels"])
    yd = torch.tensor(y, dtype=torch.float32, device=dev)
    for name, code, bound in (("f32", tfcb.F32, 1e-3), ("f16", tfcb.F16, 1e-2)):
        announce("large coarsest-grid iteration %s" % name)
        got, rep = tfcb.reconstruct(g, yd, LARGE["lam"], [1], LARGE["cgls_steps"],
                                    LARGE["framelet_levels"], storage=code)
        v = got.cpu().numpy().astype(np.float64)
        assert np.all(np.isfinite(v))
        e = float(np.linalg.norm(v - want) / np.linalg.norm(want))
        print("large coarsest grid, one outer iteration, %s storage: rel L2 vs FP64 oracle %.3e,"
              " max abs %.3e; resid2 GPU %.6e oracle %.6e"
              % (name, e, float(np.abs(v - want).max()), rep["resid2_last"],
                 orep["resid2_last"]), flush=True)
        assert e <= bound, (name, e)
