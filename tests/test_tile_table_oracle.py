"""The batched launch's work list as recomputed by the oracle, against the
properties its definition fixes (CPU only)."""
import numpy as np

import oracle as O
import testgen


def test_tile_table_properties():
    lat = testgen.batch_lattices(64)
    vols = [testgen.volume(d) for d, _ in lat]
    precs = [O.C12 if c else O.F64 for _, c in lat]
    for T in (256, 1000, 4096):
        starts, rows = O.tile_table(vols, T, precs)
        counts = [-(-v // T) for v in vols]
        assert starts == [0] + list(np.cumsum(counts)[:-1])
        assert len(rows) == sum(counts)
        covered = [np.zeros(v, dtype=np.int32) for v in vols]
        for lat_i, first, cnt, p in rows:
            assert 0 < cnt <= T and first % T == 0 and p == precs[lat_i]
            covered[lat_i][first:first + cnt] += 1
        assert all(np.all(c == 1) for c in covered)
