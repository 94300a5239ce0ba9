"""The seeded input generators are deterministic and produce inputs of the stated structure."""
import numpy as np

import rwsynth


def test_deterministic_and_structured():
    w = rwsynth.CFG1
    J1, r1 = rwsynth.phantom(w)
    J2, r2 = rwsynth.phantom(w)
    np.testing.assert_array_equal(J1, J2)
    n1, l1 = rwsynth.seeds(w, r1)
    n2, l2 = rwsynth.seeds(w, r2)
    np.testing.assert_array_equal(n1, n2)
    np.testing.assert_array_equal(l1, l2)
    assert J1.shape == (64 * 64,)
    assert np.all(np.diff(n1) > 0)                       # sorted, no duplicates
    lab = rwsynth.label_map(r1, w.C)
    np.testing.assert_array_equal(lab[n1], l1)           # seeds carry their ground-truth label
    assert np.bincount(l1).min() >= w.seeds_per_label
    # noise level as stated
    bg = r1 == 0
    assert abs(np.std(J1[bg]) - w.sigma) < 0.01


def test_cfg2_edits():
    e = rwsynth.cfg2_edits(rwsynth.CFG2)
    assert [x.kind for x in e] == ["set_beta", "scale_box", "remove_edges"]
    assert e[0].value == 150.0
    lo, hi = e[1].box_lo, e[1].box_hi
    assert hi[0] - lo[0] == 32 and hi[1] - lo[1] == 32 and 0 <= lo[0] <= 480 and 0 <= lo[1] <= 480
    ids = e[2].edge_ids
    assert ids.size == 500 and np.unique(ids).size == 500
    assert np.all(np.isin(ids, rwsynth.edge_ids_valid(rwsynth.CFG2.dims, 8)))


def test_cfg4_ragged():
    imgs = rwsynth.cfg4_images(8)
    assert all(128 <= w.dims[0] <= 768 and 128 <= w.dims[1] <= 768 for w in imgs)
    assert all(w.m in (50, 100, 200) for w in imgs)
