"""Seeded input generators: the R-MAT recipe of the skewed-degree workload
(edges i < j, no self loops or duplicates, deterministic per seed, heavy-tailed
degrees) and the matrix completion sample count."""

import numpy as np

import gen


def test_rmat_recipe():
    g = gen.rmat_graph(12, 8, 41, "gauss")
    h = gen.rmat_graph(12, 8, 41, "gauss")
    assert g.n == 4096
    assert np.array_equal(g.ei, h.ei) and np.array_equal(g.ej, h.ej) and np.array_equal(g.w, h.w)
    assert np.all(g.ei < g.ej) and g.ei.min() >= 0 and g.ej.max() < g.n
    keys = g.ei.astype(np.int64) * g.n + g.ej
    assert np.unique(keys).size == keys.size and np.all(np.diff(keys) > 0)   # sorted, no duplicates
    assert g.m_edges <= 8 * g.n
    deg = np.bincount(np.concatenate([g.ei, g.ej]), minlength=g.n)
    assert deg.max() >= 20 * deg.mean()                                      # heavy-tailed degrees
    other = gen.rmat_graph(12, 8, 42, "gauss")
    other_keys = other.ei.astype(np.int64) * other.n + other.ej
    assert other_keys.size != keys.size or not np.array_equal(other_keys, keys)   # another seed, another graph


def test_completion_sample_count_matches_the_recipe():
    inst = gen.completion_instance(500, 500, 3, 1)
    n, r = 1000, 3
    assert inst.m == gen.sample_count(500, 500, 3)
    assert inst.m == int(np.ceil(r * np.log(n) * r * (n - r)))
