"""The C-ABI library on the host (no GPU needed): it loads, exports every
symbol include/tfcb.h declares, sizes workspaces, and rejects bad arguments
before touching the device."""
import ctypes
import dataclasses
import os
import re

import numpy as np
import pytest

from paper_1008_2042_amd import inputs, tfcb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    if not os.path.exists(tfcb.LIB_PATH):
        pytest.skip("libtfcb.so not built (run __graft_entry__.build())")
    return tfcb.load()


def test_header_declarations_are_exported():
    lib = _lib()
    with open(os.path.join(ROOT, "include", "tfcb.h")) as fh:
        hdr = fh.read()
    declared = sorted(set(re.findall(r"\b(tfcb_[a-z_0-9]+)\s*\(", hdr)))
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(tfcb.EXPORTS) == declared


def test_version_and_status_strings():
    lib = _lib()
    assert b"gfx950" in lib.tfcb_version()
    assert lib.tfcb_status_str(0) == b"ok"
    assert lib.tfcb_status_str(-2) == b"workspace too small"


def test_workspace_sizes():
    _lib()
    g = inputs.config("paper")["geom"]
    opts = tfcb.options(5e-4, [16, 24])
    n = tfcb.workspace_size(g, opts)
    V, S = 512 * 512 * 70 * 4, 40 * 384 * 512 * 4
    # 7 volumes + 4 projection sets on the fine grid, plus the coarse grid
    assert 7 * V + 4 * S <= n <= 1.3 * (7 * V + 4 * S)
    n16 = tfcb.workspace_size(g, tfcb.options(5e-4, [16, 24], storage=tfcb.F16))
    assert n16 < 0.55 * n
    assert tfcb.operator_workspace_size(g, tfcb.F32) >= V


@pytest.mark.parametrize("field,value", [("nx", 0), ("dz", -1.0), ("sdd", 500.0), ("n_views", 0),
                                         ("sad", 100.0)])
def test_bad_geometry_rejected(field, value):
    lib = _lib()
    g = inputs.config("paper")["geom"]
    cg = tfcb.geometry(g)
    setattr(cg, field, value)
    n = ctypes.c_size_t(0)
    st = lib.tfcb_operator_workspace_size(ctypes.byref(cg), 0, ctypes.byref(n))
    assert st == tfcb.EINVAL
    assert len(lib.tfcb_last_error()) > 0
    # operator calls validate before any device work
    st = lib.tfcb_project(ctypes.byref(cg), 0, 256, 256, 256, 1 << 30, None)
    assert st == tfcb.EINVAL
    for name in ("tfcb_project_siddon", "tfcb_backproject_eq3"):
        assert getattr(lib, name)(ctypes.byref(cg), 0, 256, 256, 256, 1 << 30, None) == tfcb.EINVAL


def test_bad_options_and_workspace_rejected():
    lib = _lib()
    g = tfcb.geometry(inputs.config("tiny")["geom"])
    n = ctypes.c_size_t(0)
    for kw in (dict(lam=-1.0), dict(lam=float("nan")), dict(iters=[1, 1, 1, 1, 1]),
               dict(cgls_steps=0), dict(framelet_levels=3), dict(storage=7)):
        args = dict(lam=5e-4, iters=[10], cgls_steps=3, framelet_levels=1, storage=0)
        args.update(kw)
        o = tfcb.options(args["lam"], args["iters"][:4], args["cgls_steps"],
                         args["framelet_levels"], storage=args["storage"])
        if len(args["iters"]) > 4:
            o.n_grids = 5
        assert lib.tfcb_workspace_size(ctypes.byref(g), ctypes.byref(o), ctypes.byref(n)) \
            == tfcb.EINVAL, kw
    for pair in (-1, 2):
        o = tfcb.options(5e-4, [10], op_pair=pair)
        assert lib.tfcb_workspace_size(ctypes.byref(g), ctypes.byref(o), ctypes.byref(n)) \
            == tfcb.EINVAL, pair
    o = tfcb.options(5e-4, [10], op_pair=1)
    assert lib.tfcb_workspace_size(ctypes.byref(g), ctypes.byref(o), ctypes.byref(n)) == 0
    o = tfcb.options(5e-4, [10])
    assert lib.tfcb_workspace_size(ctypes.byref(g), ctypes.byref(o), ctypes.byref(n)) == 0
    # too small / misaligned / NULL workspace
    st = lib.tfcb_reconstruct(ctypes.byref(g), ctypes.byref(o), 256, 256, 256, n.value - 1, None,
                              None)
    assert st == tfcb.ENOMEM
    st = lib.tfcb_reconstruct(ctypes.byref(g), ctypes.byref(o), 256, 256, 257, n.value, None, None)
    assert st == tfcb.EINVAL
    st = lib.tfcb_reconstruct(ctypes.byref(g), ctypes.byref(o), None, 256, 256, n.value, None, None)
    assert st == tfcb.EINVAL


def test_framelet_argument_checks():
    lib = _lib()
    n = ctypes.c_size_t(0)
    assert lib.tfcb_framelet_workspace_size(8, 8, 8, 1, 0, ctypes.byref(n)) == 0 and n.value == 0
    assert lib.tfcb_framelet_workspace_size(8, 8, 8, 2, 0, ctypes.byref(n)) == 0 and n.value >= 4096
    assert lib.tfcb_framelet_workspace_size(8, 8, 8, 3, 0, ctypes.byref(n)) == tfcb.EINVAL
    # in == out is rejected
    assert lib.tfcb_framelet_shrink(8, 8, 8, 1, 0.1, 1, 0, 256, 256, None, 0, None) == tfcb.EINVAL


def test_product_path_does_not_reference_the_oracle():
    """The GPU package never imports, links or loads the oracle."""
    pkg = os.path.join(ROOT, "paper_1008_2042_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")) and f != "inputs.py":
                with open(os.path.join(dirpath, f)) as fh:
                    text = fh.read()
                assert "import oracle" not in text and "tf_oracle" not in text, f


def test_every_grid_of_the_schedule_is_validated():
    """Coarser grids are checked like the finest: a detector binned 2 x 2
    for the next grid must have even sizes (each coarse pixel centre is then
    the mean of the four it averages), and a coarse grid (ceil sizes, twice
    the voxel, so larger in mm) must stay inside the source orbit."""
    lib = _lib()
    n = ctypes.c_size_t(0)
    base = inputs.Geometry(48, 40, 12, 1.5, 1.5, 1.5, 96, 48, 2.0, 2.0, n_views=20)
    o2 = tfcb.options(5e-4, [2, 2])
    assert lib.tfcb_workspace_size(ctypes.byref(tfcb.geometry(base)), ctypes.byref(o2),
                                   ctypes.byref(n)) == 0
    for nu, nv in ((97, 48), (96, 47)):
        odd = inputs.Geometry(48, 40, 12, 1.5, 1.5, 1.5, nu, nv, 2.0, 2.0, n_views=20)
        assert lib.tfcb_workspace_size(ctypes.byref(tfcb.geometry(odd)), ctypes.byref(o2),
                                       ctypes.byref(n)) == tfcb.EUNSUPPORTED
        assert b"even" in lib.tfcb_last_error()
        # one grid, or no binning: nothing is binned, so odd sizes are fine
        for o in (tfcb.options(5e-4, [2]), tfcb.options(5e-4, [2, 2], bin_detector=False)):
            assert lib.tfcb_workspace_size(ctypes.byref(tfcb.geometry(odd)), ctypes.byref(o),
                                           ctypes.byref(n)) == 0
    # a fine grid just inside the orbit whose two-grid coarse grid is not:
    # fine half-diagonal (0.5*181 + 2) * 1.0 * sqrt(2) = 130.8 < 140, coarse
    # (0.5*91 + 2) * 2.0 * sqrt(2) = 134.4 ... with 3 grids (0.5*46 + 2) * 4 * sqrt(2) = 141.4
    wide = inputs.Geometry(181, 181, 8, 1.0, 1.0, 1.0, 64, 16, 1.0, 1.0, sad=140.0, sdd=210.0,
                           n_views=8)
    o1 = tfcb.options(5e-4, [2])
    assert lib.tfcb_workspace_size(ctypes.byref(tfcb.geometry(wide)), ctypes.byref(o1),
                                   ctypes.byref(n)) == 0
    o3 = tfcb.options(5e-4, [1, 1, 1])
    assert lib.tfcb_workspace_size(ctypes.byref(tfcb.geometry(wide)), ctypes.byref(o3),
                                   ctypes.byref(n)) == tfcb.EINVAL
    assert b"coarse grid 2" in lib.tfcb_last_error()


def test_tv_options_and_rof_arguments_checked():
    lib = _lib()
    g = tfcb.geometry(inputs.config("tiny")["geom"])
    n = ctypes.c_size_t(0)
    ok = tfcb.options(5e-4, [10], regulariser=1)
    assert lib.tfcb_workspace_size(ctypes.byref(g), ctypes.byref(ok), ctypes.byref(n)) == 0
    tf = ctypes.c_size_t(0)
    assert lib.tfcb_workspace_size(ctypes.byref(g), ctypes.byref(tfcb.options(5e-4, [10])),
                                   ctypes.byref(tf)) == 0
    assert n.value > tf.value  # the FP32 gradient volume and descent state
    for kw in (dict(regulariser=2), dict(regulariser=1, tv_eps=0.0),
               dict(regulariser=1, tv_tol=-1.0), dict(regulariser=1, tv_max_steps=-1)):
        o = tfcb.options(5e-4, [10], **kw)
        assert lib.tfcb_workspace_size(ctypes.byref(g), ctypes.byref(o), ctypes.byref(n)) \
            == tfcb.EINVAL, kw
    assert lib.tfcb_rof_workspace_size(8, 8, 8, ctypes.byref(n)) == 0 and n.value >= 8 ** 3 * 4
    nul = ctypes.c_int32(0)
    args = (8, 8, 8, 1e-3, 1e-5, 1e-3, 100, 1, 0)
    assert lib.tfcb_rof(*args, 256, 256, 256, n.value, None, ctypes.byref(nul)) == tfcb.EINVAL
    assert lib.tfcb_rof(*args, None, 512, 256, n.value, None, ctypes.byref(nul)) == tfcb.EINVAL
    assert lib.tfcb_rof(8, 8, 8, -1.0, 1e-5, 1e-3, 100, 1, 0, 256, 512, 256, n.value, None,
                        ctypes.byref(nul)) == tfcb.EINVAL
    assert lib.tfcb_rof(*args, 256, 512, 256, n.value - 1, None, ctypes.byref(nul)) \
        == tfcb.ENOMEM


def test_geometry_size_limits_and_angles():
    """Sizes past the library's index limits and non-finite angles are
    refused before any work, with a message naming the limit."""
    lib = _lib()
    n = ctypes.c_size_t(0)
    base = inputs.config("tiny")["geom"]
    cases = [
        (dict(nz=70000), tfcb.EUNSUPPORTED, "65535"),
        (dict(nv=20000), tfcb.EUNSUPPORTED, "detector"),
        # 2^31 voxels
        (dict(nx=2048, ny=2048, nz=600, dx=0.01, dy=0.01, dz=0.01), tfcb.EUNSUPPORTED, "2^31"),
        # the padded copy alone exceeds 2^31 elements: (nz + 12) * 4096 * 4100
        (dict(nx=4096, ny=4096, nz=120, dx=0.01, dy=0.01, dz=0.01), tfcb.EUNSUPPORTED,
         "padded"),
    ]
    for kw, want, word in cases:
        g = tfcb.geometry(dataclasses.replace(base, **kw))
        st = lib.tfcb_operator_workspace_size(ctypes.byref(g), 0, ctypes.byref(n))
        assert st == want, (kw, st)
        assert word in lib.tfcb_last_error().decode(), (kw, lib.tfcb_last_error())
    ang = np.linspace(0.0, 6.0, base.n_views)
    ang[3] = float("inf")
    g = tfcb.geometry(dataclasses.replace(base, angles=ang))
    assert lib.tfcb_operator_workspace_size(ctypes.byref(g), 0, ctypes.byref(n)) == tfcb.EINVAL
    assert "angle 3" in lib.tfcb_last_error().decode()


def test_fdk_arguments_checked():
    """FDK assumes the circular orbit's uniform angles and a row that fits its
    filter's LDS staging; both are checked on the host before any work."""
    lib = _lib()
    n = ctypes.c_size_t(0)
    base = inputs.config("tiny")["geom"]
    g = tfcb.geometry(base)
    assert lib.tfcb_fdk_workspace_size(ctypes.byref(g), ctypes.byref(n)) == 0
    assert n.value >= base.n_views * base.nv * base.nu * 4
    g = tfcb.geometry(dataclasses.replace(base, angles=np.linspace(0.0, 6.0, base.n_views)))
    assert lib.tfcb_fdk(ctypes.byref(g), 0, 256, 256, 256, 1 << 30, None) == tfcb.EUNSUPPORTED
    assert "angles" in lib.tfcb_last_error().decode()
    g = tfcb.geometry(dataclasses.replace(base, nu=9000, du=0.01))
    assert lib.tfcb_fdk(ctypes.byref(g), 0, 256, 256, 256, 1 << 30, None) == tfcb.EUNSUPPORTED
    assert "8192" in lib.tfcb_last_error().decode()
