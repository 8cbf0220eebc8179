"""The continuous-batching server: every result equals the same request's
standalone reconstruction bit for bit, alone or in a mix; admission by HBM
budget; failure isolation; cancellation."""
import sys

import numpy as np
import pytest

from paper_1008_2042_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1008_2042_amd import serve, tfcb  # noqa: E402


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def announce(msg):
    print("[gpu-case]", msg, flush=True)
    sys.stdout.flush()


def _requests(dev):
    """Four small requests of different shapes, schedules and storage types."""
    specs = [
        (inputs.Geometry(64, 64, 16, 1.0, 1.0, 1.0, 128, 64, 1.5, 1.5, n_views=30), 101,
         dict(iters=[4]), tfcb.F32),
        (inputs.serving_geometry(128, 128, 20), 4001, dict(iters=[3, 2]), tfcb.F16),
        (inputs.Geometry(48, 40, 12, 1.5, 1.5, 1.5, 96, 48, 2.0, 2.0, n_views=20), 7,
         dict(iters=[2, 3], framelet_levels=2), tfcb.F32),
        (inputs.serving_geometry(128, 128, 40), 4002, dict(iters=[2, 2]), tfcb.BF16),
    ]
    out = []
    for g, seed, kw, storage in specs:
        ells = inputs.tiny_phantom(seed) if g.nx <= 64 else inputs.body_phantom(seed, 4, 15)
        y = inputs.analytic_projection_torch(g, ells, dev).to(torch.float32).contiguous()
        opts = tfcb.options(5e-4, kw["iters"], 3, kw.get("framelet_levels", 1), storage=storage)
        out.append(dict(geom=g, proj=y, opts=opts, kw=kw, storage=storage,
                        bytes=tfcb.Server.request_bytes(g, opts)))
    return out


def _alone(r):
    vol, _ = tfcb.reconstruct(r["geom"], r["proj"], 5e-4, r["kw"]["iters"],
                              framelet_levels=r["kw"].get("framelet_levels", 1),
                              storage=r["storage"])
    return vol.clone()


def test_mix_equals_alone_bitwise():
    dev = _dev()
    reqs = _requests(dev)
    announce("serving alone")
    alone = [_alone(r) for r in reqs]
    announce("serving mix")
    arena = 2 * sum(r["bytes"] for r in reqs)
    run = serve.replay(reqs, np.zeros(len(reqs)), arena, max_slots=4, keep_results=True)
    for i, r in enumerate(reqs):
        assert run["status"][i][0] == tfcb.REQ_DONE, run["status"][i]
        assert torch.equal(run["results"][i], alone[i]), i
    assert np.all(run["latency"] > 0)
    # staggered arrivals: the same results again
    announce("serving staggered")
    run2 = serve.replay(reqs, np.array([0.0, 0.01, 0.02, 0.05]), arena, max_slots=2,
                        keep_results=True)
    for i in range(len(reqs)):
        assert torch.equal(run2["results"][i], alone[i]), i


def test_budget_admits_one_at_a_time():
    dev = _dev()
    reqs = _requests(dev)[:3]
    alone = [_alone(r) for r in reqs]
    arena = max(r["bytes"] for r in reqs) + 4096
    announce("serving tight budget")
    run = serve.replay(reqs, np.zeros(len(reqs)), arena, max_slots=4, keep_results=True)
    for i in range(len(reqs)):
        assert run["status"][i][0] == tfcb.REQ_DONE
        assert torch.equal(run["results"][i], alone[i])
    # one at a time: completion order follows submission order
    assert np.all(np.diff(run["latency"]) > 0)


def test_too_large_request_rejected():
    dev = _dev()
    r = _requests(dev)[0]
    srv = tfcb.Server(r["bytes"] // 2, 2)
    with pytest.raises(tfcb.TfcbError) as ei:
        srv.submit(r["geom"], r["proj"], r["opts"])
    assert ei.value.status == tfcb.ENOMEM
    srv.close()


def test_tv_request_refused():
    """The server runs the tight-frame method only; a TV request is refused
    at submission."""
    dev = _dev()
    r = _requests(dev)[0]
    srv = tfcb.Server(r["bytes"] * 2, 2)
    o = tfcb.options(5e-4, [2], storage=tfcb.F16, regulariser=1)
    with pytest.raises(tfcb.TfcbError) as ei:
        srv.submit(r["geom"], r["proj"], o)
    assert ei.value.status == tfcb.EUNSUPPORTED
    srv.close()


def test_nan_request_fails_alone():
    dev = _dev()
    reqs = _requests(dev)[:3]
    alone = [_alone(r) for r in reqs]
    bad = dict(reqs[1])
    p = bad["proj"].clone()
    p[0, 5, 7] = float("nan")
    bad["proj"] = p
    mix = [reqs[0], bad, reqs[2]]
    announce("serving nan")
    run = serve.replay(mix, np.zeros(3), 2 * sum(r["bytes"] for r in mix), 4, keep_results=True)
    assert run["status"][1] == (tfcb.REQ_FAILED, tfcb.ENUMERIC)
    assert torch.equal(run["results"][0], alone[0])
    assert torch.equal(run["results"][2], alone[2])


def test_cancel_running_request():
    dev = _dev()
    reqs = _requests(dev)[:2]
    srv = tfcb.Server(2 * sum(r["bytes"] for r in reqs), 2)
    ids = [srv.submit(r["geom"], r["proj"], r["opts"]) for r in reqs]
    announce("serving cancel")
    srv.step()
    srv.step()
    srv.cancel(ids[1])
    assert srv.poll(ids[1])[0] == tfcb.REQ_CANCELLED
    for _ in range(10000):
        srv.step()
        if srv.poll(ids[0])[0] == tfcb.REQ_DONE:
            break
    assert srv.poll(ids[0])[0] == tfcb.REQ_DONE
    assert torch.equal(srv.result(ids[0]), _alone(reqs[0]))
    srv.close()
