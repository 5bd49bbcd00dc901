"""Host checks of the generated 7x7 median networks (no GPU): the generator
proves every network on all 0-1 inputs with sorted lists and checks the
composed four-window step against numpy's median on random inputs with ties
before it writes the include file."""

import importlib.util
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
GEN = os.path.join(HERE, "..", "paper_2307_12988_amd", "csrc", "gen_median_net.py")


def _gen():
    spec = importlib.util.spec_from_file_location("gen_median_net", GEN)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_generator_checks_pass_and_file_matches_checked_in(tmp_path):
    g = _gen()
    out = tmp_path / "net.inc"
    assert g.main(str(out)) == 0
    with open(os.path.join(HERE, "..", "paper_2307_12988_amd", "csrc", "median49_net.inc")) as fh:
        assert out.read_text() == fh.read()


def test_row_sort_sorts_every_input_with_ties():
    g = _gen()
    ops, outs = g.sort7_ops()
    rng = np.random.default_rng(4)
    v = rng.integers(0, 4, size=(50000, 7)).astype(np.float64)
    assert np.array_equal(g.evaluate(ops, outs, v), np.sort(v, axis=1))
    assert len(ops) == 27  # 25 instructions once min(min()) and max(max()) fuse


def test_row_median_is_the_fourth_smallest_with_ties():
    g = _gen()
    ops, outs = g.med7_ops()
    rng = np.random.default_rng(5)
    for v in (rng.integers(0, 4, size=(50000, 7)).astype(np.float64), rng.random((50000, 7))):
        assert np.array_equal(g.evaluate(ops, outs, v)[:, 0], np.sort(v, axis=1)[:, 3])
    assert len(ops) == 15  # 13 instructions once min(min()) and max(max()) fuse


def test_window_median_lies_between_its_row_medians():
    """The bound the centre-only start relies on: a 7x7 window's median is
    at least the smallest and at most the largest median of its rows."""
    rng = np.random.default_rng(6)
    for v in (rng.integers(0, 3, size=(20000, 7, 7)).astype(np.float64),
              rng.random((20000, 7, 7)) ** 3):
        med = np.sort(v.reshape(-1, 49), axis=1)[:, 24]
        rows = np.sort(v, axis=2)[:, :, 3]
        assert np.all(rows.min(axis=1) <= med) and np.all(med <= rows.max(axis=1))


def test_med3_rewrite_keeps_the_merge_and_saves_operations():
    g = _gen()
    for lens, ranks in (([22, 14], list(range(14, 22))), ([14, 14], list(range(3, 25))),
                        ([8, 7], [7])):
        kept, outs = g.merge_select(lens, ranks)
        fused = g.fuse_med3(kept, outs, lens)
        assert len(fused) < len(kept)
        g.check_zero_one(fused, outs, lens, ranks)
        rng = np.random.default_rng(len(kept))
        v = np.concatenate([np.sort(rng.integers(0, 6, size=(20000, n)), axis=1) for n in lens],
                           axis=1).astype(np.float64)
        assert np.array_equal(g.evaluate(fused, outs, v), np.sort(v, axis=1)[:, ranks])


def test_med3_rewrite_is_refused_without_the_order_fact():
    """max(min(a, b), c) is a med3 only when c <= a or c <= b is known: on two
    free inputs lists of length one nothing is known, so nothing is fused."""
    g = _gen()
    kept = [(3, "min", 0, 1), (4, "max", 3, 2)]
    assert g.fuse_med3(kept, [4], [1, 1, 1]) == kept


def test_med3_rewrite_applies_with_the_order_fact():
    """Inputs 0 <= 1 (one sorted list) and a free input 2: max(min(x1, x2), x0)
    becomes med3(x1, x2, x0), which equals it on every input."""
    g = _gen()
    kept = [(3, "min", 1, 2), (4, "max", 3, 0)]
    fused = g.fuse_med3(kept, [4], [2, 1])
    assert fused == [(4, "med3", 1, 2, 0)]
    rng = np.random.default_rng(9)
    v = rng.integers(0, 5, size=(5000, 3)).astype(np.float64)
    v[:, :2] = np.sort(v[:, :2], axis=1)
    assert np.array_equal(g.evaluate(fused, [4], v), g.evaluate(kept, [4], v))
