"""Seeded input generator: published SplitMix64 test vector, normal
statistics, and the planted-partition graph recipe."""
import numpy as np

import abg_synth as s


def test_splitmix64_published_vector():
    # first outputs of SplitMix64 from state 1234567 (Steele et al. reference
    # implementation test vector)
    st = 1234567
    out = []
    for _ in range(5):
        st, z = s._splitmix64_next(st)
        out.append(z)
    assert out == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                   4593380528125082431, 16408922859458223821]


def test_normals_statistics_and_determinism():
    a = s.splitmix64_normals(42, 1, 200_001)
    b = s.splitmix64_normals(42, 1, 200_001)
    assert np.array_equal(a, b)
    assert abs(a.mean()) < 0.01 and abs(a.var() - 1) < 0.01
    c = s.splitmix64_normals(42, 2, 1000)
    assert not np.allclose(a[:1000], c)
    # prefix property: a shorter draw is a prefix of a longer one
    assert np.array_equal(s.splitmix64_normals(42, 1, 7), a[:7])


def test_method_matrix_shapes():
    mm = s.method_matrices(0, 256, 64, 20)
    assert mm.omega_reduce.shape == (256, 74)
    assert mm.g.shape == (64, 64)
    assert mm.omega.shape == (128, 30)
    mm = s.method_matrices(0, 64, 0, 5)
    assert mm.omega_reduce is None and mm.g.shape == (64, 64) and mm.omega.shape == (128, 15)
    assert s.sketch_widths(16, 8, 20, 10) == (8, 16, 16)


def test_planted_graph_recipe():
    g = s.planted_abg(3000, 4000, 30_000, 6, 12, zipf_a=2.0, seed=5)
    assert g.n_edges == 30_000
    key = g.edge_u.astype(np.int64) * g.n_v + g.edge_v
    assert np.unique(key).size == key.size
    assert g.edge_u.dtype == np.int32 and g.x_u.dtype == np.float32
    assert np.bincount(g.labels_u, minlength=6).min() == 500
    intra = (g.labels_u[g.edge_u] == g.labels_v[g.edge_v]).mean()
    # draws are 8/(8+k-1) intra-cluster; dropping repeated pairs (mostly hub
    # pairs inside a cluster) lowers the kept fraction somewhat, far above 1/k
    assert 0.45 < intra <= 8 / (8 + 5) + 0.01
    g2 = s.planted_abg(3000, 4000, 30_000, 6, 12, zipf_a=2.0, seed=5)
    assert np.array_equal(g.edge_u, g2.edge_u) and np.array_equal(g.x_u, g2.x_u)
