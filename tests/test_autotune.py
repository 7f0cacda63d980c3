"""Host logic of the tile-shape tuner (no GPU): the cache key ignores the tile width and
nothing else, and models below the tuner's tile threshold keep the default shape untimed."""
import pytest

import workloads as W

torch = pytest.importorskip("torch")

from paper_2608_23245_amd import autotune as A  # noqa: E402
from paper_2608_23245_amd import binding as B  # noqa: E402


def test_model_key_ignores_only_the_tile_width():
    m = B.make_model(W.config1())
    k = A.model_key(m, 100)
    assert A.model_key(A.with_tile_w(m, 16), 100) == k
    assert A.with_tile_w(m, 16).geom.tile_w == 16 and m.geom.tile_w == 0
    assert A.model_key(m, 101) != k
    for change in (lambda x: setattr(x.geom, "width", 1000), lambda x: setattr(x.dis, "sigma_theta", 0.1),
                   lambda x: setattr(x.quad, "n_nodes", 32), lambda x: setattr(x.cell, "a", 41.0)):
        m2 = B.Model.from_buffer_copy(m)
        change(m2)
        assert A.model_key(m2, 100) != k


def test_candidates_must_include_the_default():
    with pytest.raises(ValueError):
        A.TileTuner(candidates=(4, 16))


def test_small_models_keep_the_default_untimed():
    """Below min_tiles the tuner times nothing (no launch) and caches the default."""
    m = B.make_model(W.config1())
    t = A.TileTuner(min_tiles=10 ** 9)
    refl = torch.zeros((7, B.REFL_FLOATS), dtype=torch.float32)
    assert t.choose(m, refl, None, None) == A.DEFAULT
    assert t.cached(A.with_tile_w(m, 16), 7) == (A.DEFAULT, {})
    assert t.cached(m, 8) is None
