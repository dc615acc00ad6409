"""Base-2 accumulation storage (appendix A.4, binary storage system, fig. St):
rebuilt estimates are plain means over the source subsets the binary digits
of n select."""
import numpy as np
import pytest

from paper_1309_2256_amd.storage import Base2Store


def sources(n, shape=(2, 3, 16, 4), seed=0):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal(shape) + 1j * rng.standard_normal(shape) for _ in range(n)]


def test_figure_example_thirteen_of_fifteen():
    """The paper's example: 13 = 1 + 4 + 8 uses File.1, File.4 and File.8,
    i.e. source 1 and sources 4 .. 15."""
    xs = sources(15)
    st = Base2Store(xs[0].shape)
    st.add_many(xs)
    assert st.counts == [1, 2, 4, 8] and len(st.sums) == 4
    assert st.sources(13) == [1] + list(range(4, 16))
    want = (xs[0] + sum(xs[3:15])) / 13
    assert np.abs(st.mean(13) - want).max() < 1e-14


@pytest.mark.parametrize("n_added", [1, 2, 7, 8, 20, 63])
def test_every_reachable_n_is_a_subset_mean(n_added):
    xs = sources(n_added, seed=n_added)
    st = Base2Store(xs[0].shape)
    st.add_many(xs)
    assert len(st.sums) == n_added.bit_length()      # O(log2 N) stored arrays
    assert np.abs(sum(st.sums) - sum(xs)).max() < 1e-12
    for n in range(1, st.max_reachable() + 1):
        idx = [i - 1 for i in st.sources(n)]
        assert len(idx) == n
        assert np.abs(st.mean(n) - sum(xs[i] for i in idx) / n).max() < 1e-13
    if st.max_reachable() < n_added:
        with pytest.raises(ValueError):
            st.total(1 << (len(st.sums) - 1))           # the incomplete top bin


def test_save_load_round_trip(tmp_path):
    xs = sources(11, shape=(3, 5, 16, 8), seed=3)
    st = Base2Store(xs[0].shape)
    st.add_many(xs)
    st.save(tmp_path, "std")
    assert sorted(p.name for p in tmp_path.iterdir()) == \
        ["std.1.npy", "std.2.npy", "std.4.npy", "std.8.npy", "std.index.json"]
    back = Base2Store.load(tmp_path, "std")
    assert back.counts == st.counts and back.n == 11
    for a, b in zip(back.sums, st.sums):
        assert np.array_equal(a, b)
    assert np.array_equal(back.mean(7), st.mean(7))


def test_rejects_wrong_shape_and_n():
    st = Base2Store((16, 4))
    with pytest.raises(ValueError):
        st.add(np.zeros((16, 5)))
    with pytest.raises(ValueError):
        st.mean(0)
