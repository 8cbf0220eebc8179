"""The image-quality protocols of section 3.2 (MTF from a 0.28 mm bead, CNR
against the threshold, a 200-degree short scan) run end to end on the GPU at
paper scale.  They measure, they do not pin: the assertions are sanity
checks of the measurement itself (an MTF that starts at 1 and falls, CNR
values that are finite and positive, errors below 100 %)."""
import json

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.timeout(600)
def test_quality_protocols_run():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1008_2042_amd import quality
    res = quality.run(torch.device("cuda:0"))
    print(json.dumps(res), flush=True)
    for name, m in res["mtf"].items():
        curve = np.array(m["mtf"])
        assert curve[0] == pytest.approx(1.0) and curve[-1] < 1.0, name
        assert 0.0 < m["mtf50_cycles_per_mm"] <= res["mtf_frequencies_cycles_per_mm"][-1], name
    cnr = [s["cnr_bone_mean"] for s in res["cnr_vs_lambda"]]
    assert all(np.isfinite(cnr)) and min(cnr) > 0
    assert 0.0 < res["rrms_in_body_tf"]["full_360"] < 1.0
    assert 0.0 < res["rrms_in_body_tf"]["short_200"] < 1.0
