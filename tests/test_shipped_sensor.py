"""The shipped sensor network (paper_2007_14933_amd/sensor_weights.npz): its
shape and the training recipe it records.  Host only."""
import os

import numpy as np

from paper_2007_14933_amd import sensor as SN


def test_shipped_weights_and_recipe():
    assert os.path.exists(SN.DEFAULT_WEIGHTS)
    d = np.load(SN.DEFAULT_WEIGHTS, allow_pickle=False)
    w = d["weights_bf16"]
    # 10 -> 32 -> 32 -> 1 with biases
    assert w.shape == (10 * 32 + 32 + 32 * 32 + 32 + 32 + 1,) == (SN.NPARAM,)
    # bfloat16 bit patterns of finite values (exponent field not all ones)
    assert np.all((w.astype(np.uint32) >> 7 & 0xFF) != 0xFF)
    assert 0.0 < float(d["threshold"]) < 1.0
    assert int(d["dilate"]) in (1, 2)
    # trained on at least 1e7 method-made labels
    assert int(d["samples"]) >= 10_000_000
    # the routing it was shipped with met the 1e-4 density bar on its held-out fields
    assert float(d["heldout_rel_L1_rho"]) <= 1e-4
