"""Host logic of the three-stage search (Sec. III.B): the boxes each stage of
fstat_search searches, against the plain restatement in oracle/search_oracle.py
(no device call is made)."""
import os

import numpy as np
import pytest

from oracle import search_oracle as SO

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
YEAR = 365.25 * 86400.0


def _lib():
    from paper_2407_10797_amd import fstat
    if not os.path.exists(fstat.LIB_PATH):
        pytest.skip("libfstat.so not built")
    return fstat


def _cfg(box, **kw):
    c = dict(box=box, n_slices=24, runs=(24, 8, 48), iters=(8000, 8000, 15000), np=(16, 16, 1),
             n_part=128, ring_k=1, w=(0.9, 0.4), c1=2.0, c2=2.0, vmax=0.5,
             width2=(0.01 * YEAR, 0.6), width3=(0.004 * YEAR, 0.3, 0.4, 0.4, 0.006), seed=7)
    c.update(kw)
    return c


PAPER_BOX = np.array([[3.3 * YEAR, 3.8 * YEAR], [10.0, 50.0], [0.0, 0.9], [0.0, np.pi],
                      [0.0, 2 * np.pi], [0.0, 0.1]])


def _desc(fstat, cfg):
    keys = ("n_slices", "runs", "iters", "np", "n_part", "ring_k", "w", "c1", "c2", "vmax",
            "width2", "width3")
    return fstat.search_desc(cfg["box"], seed=cfg["seed"], **{k: cfg[k] for k in keys})


@pytest.mark.parametrize("box", [PAPER_BOX, PAPER_BOX * [[1, 1], [1, 1], [1, 1], [1, 1], [0.5, 0.5], [1, 1]]])
def test_stage_boxes_match_reference(box):
    fstat = _lib()
    cfg = _cfg(box)
    d = _desc(fstat, cfg)
    b1 = fstat.search_boxes(d, 1)
    np.testing.assert_array_equal(b1, SO.boxes(cfg, 1))
    assert b1.shape == (24, 6, 2)
    # contiguous equal t_c intervals covering the range; other ranges full
    np.testing.assert_array_equal(b1[1:, 0, 0], b1[:-1, 0, 1])
    assert b1[0, 0, 0] == box[0, 0] and b1[-1, 0, 1] == box[0, 1]
    np.testing.assert_allclose(np.diff(b1[:, 0], axis=1), (box[0, 1] - box[0, 0]) / 24, rtol=1e-12)
    rng = np.random.default_rng(3)
    # centres: interior points and ones at the edges of the full box
    cen = box[:, 0] + rng.uniform(0, 1, (24, 6)) * (box[:, 1] - box[:, 0])
    cen[0] = box[:, 0]
    cen[1] = box[:, 1]
    b2 = fstat.search_boxes(d, 2, cen)
    np.testing.assert_array_equal(b2, SO.boxes(cfg, 2, cen))
    assert np.all(b2[:, 0, 1] - b2[:, 0, 0] <= 0.01 * YEAR * (1 + 1e-15))
    for k in range(3):
        b3 = fstat.search_boxes(d, 3, cen[k])
        np.testing.assert_array_equal(b3, SO.boxes(cfg, 3, cen[k:k + 1]))
        np.testing.assert_array_equal(b3[:, 2], np.repeat(box[None, 2], 2, axis=0))
        # the second box is centred on pi - theta (up to clipping)
        mid = 0.5 * (b3[:, 3, 0] + b3[:, 3, 1])
        if 0.2 < cen[k, 3] < np.pi - 0.2:
            np.testing.assert_allclose(mid, [cen[k, 3], np.pi - cen[k, 3]], rtol=1e-12)


def test_phi_is_not_clipped_on_the_full_circle():
    fstat = _lib()
    cfg = _cfg(PAPER_BOX)
    d = _desc(fstat, cfg)
    c = np.array([3.5 * YEAR, 30.0, 0.5, 1.0, 0.1, 0.05])
    b3 = fstat.search_boxes(d, 3, c)
    np.testing.assert_allclose(b3[0, 4], [0.1 - 0.2, 0.1 + 0.2], rtol=1e-12)
    half = PAPER_BOX.copy()
    half[4] = [0.0, np.pi]
    cfg2 = _cfg(half)
    b3h = fstat.search_boxes(_desc(fstat, cfg2), 3, c)
    np.testing.assert_allclose(b3h[0, 4], [0.0, 0.3], rtol=1e-12)
    np.testing.assert_array_equal(b3h, SO.boxes(cfg2, 3, c[None]))


def test_search_descriptor_errors():
    fstat = _lib()
    cfg = _cfg(PAPER_BOX)
    for bad in (dict(n_slices=0), dict(runs=(0, 8, 48)), dict(n_part=2000),
                dict(width2=(0.0, 0.6)), dict(width3=(1.0, 0.3, -0.4, 0.4, 0.006))):
        c = dict(cfg, **bad)
        with pytest.raises(fstat.FstatError):
            fstat.search_boxes(_desc(fstat, c), 1)
    d = _desc(fstat, cfg)
    with pytest.raises(fstat.FstatError):
        fstat.search_boxes(d, 2, None)
    with pytest.raises(fstat.FstatError):
        fstat.search_boxes(d, 4, np.zeros(6))
