"""CPU checks of the seeded input generators used by the benchmark's
comparisons: scribble labels mark every object and some background, never
with the wrong class."""

import numpy as np

from synth.graphs import rectangles_image, scribble_labels


def test_scribbles_mark_each_object_with_its_class():
    rng = np.random.default_rng(3)
    img, truth = rectangles_image(200, 240, 5, rng, side=(20, 80), noise=0.01)
    lab = scribble_labels(truth, np.random.default_rng(4)).reshape(truth.shape)
    marked = lab >= 0
    assert np.array_equal(lab[marked], truth[marked])          # right class everywhere
    from scipy import ndimage
    comps, ncomp = ndimage.label(truth == 1)
    for c in range(1, ncomp + 1):
        assert (lab[comps == c] == 1).any()                     # every object has a stroke
    assert (lab == 0).sum() >= 4 * 3 * 8                        # four background strokes
    assert marked.mean() < 0.05                                 # sparse, as scribbles are
    again = scribble_labels(truth, np.random.default_rng(4)).reshape(truth.shape)
    assert np.array_equal(lab, again)                           # seeded
