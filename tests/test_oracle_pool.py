"""The slab-parallel run of the oracle (oracle/pool.py) reproduces the serial
run exactly: Alg. 1 is block-local (blocks of 4^d values decode
independently, Sec. 6.1), so slabs cut on chunk boundaries give the same
chunk payloads, and the joined streams, measured errors and partial sums
equal one serial run byte for byte."""
import numpy as np

from oracle import driver, pool
from paper_2308_11759_amd import inputs


def test_slab_planes_cut_on_chunk_boundaries():
    for shape in ((40, 6, 10), (20, 13, 30), (512, 512, 512), (256, 256, 256), (9, 10, 11), (17, 5, 3)):
        p = pool.slab_planes(shape)
        nbx, nby = (shape[2] + 3) // 4, (shape[1] + 3) // 4
        assert p % 4 == 0 and (p // 4) * nbx * nby % 16 == 0
    assert pool.slab_planes((512, 512, 512)) == 4


def test_pooled_run_equals_serial_run():
    cases = [((20, 13, 30), np.float32, 51, [2.0 ** -3 * k for k in (1.0, 0.125, 0.015625)]),
             ((40, 6, 10), np.float64, 52, [0.1, 0.01, 0.001, 1e-4]),
             ((9, 10, 11), np.float32, 53, [0.05, 0.001])]
    for shape, dt, seed, taus in cases:
        x = inputs.spectral_field(shape, seed=seed, dtype=dt)
        comps, meta = driver.compress(x, taus)
        pc, pm, precon = pool.compress(x, taus, workers=3)
        for i in range(len(taus)):
            assert bytes(pc[i]) == bytes(comps[i]), (shape, i)
            assert pm[i]["linf"] == meta[i]["linf"]
            for key in ("nempty", "ncoded", "nraw", "nesc", "nmiss"):
                assert pm[i][key] == meta[i][key]
            assert np.array_equal(precon[i], driver.reconstruct(comps, i + 1, x.shape, x.dtype))
    # more than one slab really ran in the first two cases
    assert len(pool.slabs((20, 13, 30), pool.slab_planes((20, 13, 30)))) == 5
    assert len(pool.slabs((40, 6, 10), pool.slab_planes((40, 6, 10)))) == 2
