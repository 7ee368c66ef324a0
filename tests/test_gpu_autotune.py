"""GPU check of the autotuner: it returns options that keep parity, caches
them, and a plan built from the cache matches the oracle."""
import json

import numpy as np
import pytest

from nudft import rel_l2
from paper_1710_03197_amd import data

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_autotune_roundtrip(orc, tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1710_03197_amd import autotune
    dev = torch.device("cuda:0")
    c = data.config1()
    N, K, J, om = c["N"], c["K"], c["J"], c["om"]
    path = str(tmp_path / "tune.json")
    om_t = torch.from_numpy(om).to(dev)
    res = autotune.tune(om_t, N, K, J, reps=3, path=path)
    print("tuned:", res, flush=True)
    assert res["tried"] >= 10
    assert set(res["options"]) >= {"tile", "grid_chunk", "fft_groups"}
    db = json.load(open(path))
    assert autotune.workload_key(N, K, J, om.shape[0]) in db
    p = autotune.tuned_plan(om_t, N, K, J, path=path)
    assert p.options == autotune.cached_options(N, K, J, om.shape[0], path)
    y = p.forward(torch.from_numpy(c["x"]).to(dev)).cpu().numpy()
    assert rel_l2(y, orc.forward(c["x"], om, N, K, J)) < 1e-5
    p.close()
