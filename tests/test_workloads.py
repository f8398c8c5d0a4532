"""Input generators: counts, density, slab split, RSA minimum distance, seeding."""
import numpy as np
from scipy.spatial import cKDTree

import workloads as W


def test_wurtzite_counts_and_box():
    pos, sp, box = W.wurtzite_ideal(40, 20, 15)
    assert pos.shape == (96000, 3)
    assert np.allclose(box, [127.6, 110.50484152, 77.85])
    assert (sp == 0).sum() == (sp == 1).sum()


def test_slab_split_and_rsa_distance():
    d = W.wurtzite_slab(6, 4, 6, seed=3)
    pos, box = d["pos"].astype(np.float64), d["box"]
    n = pos.shape[0]
    assert n == 6 * 4 * 6 * 8 and int(d["n_crystal"]) == n // 2
    rnd = pos[int(d["n_crystal"]):]
    assert np.all(rnd[:, 2] >= box[2] / 2 - 1e-5)
    # every random atom is >= 1.6 A from every other atom (periodic)
    tree = cKDTree(np.mod(pos, box), boxsize=box)
    dd, _ = tree.query(rnd, k=2)
    assert np.all(dd[:, 1] >= 1.6 - 1e-5)
    assert np.all((pos >= 0) & (pos < box))


def test_seeded_and_float32():
    a = W.wurtzite_slab(4, 3, 4, seed=31)
    b = W.wurtzite_slab(4, 3, 4, seed=31)
    assert a["pos"].dtype == np.float32 and np.array_equal(a["pos"], b["pos"])
    f = W.fcc_jittered()
    assert f["pos"].shape == (864, 3)


def test_hill_centres_range():
    c = W.hill_centres(1000, [0.0], [14.0], seed=11)
    assert c.shape == (1000, 1) and c.min() >= 0 and c.max() < 14

