"""The seeded SU(3) input generator (CPU only)."""
import numpy as np

import testgen
from pins import to_complex


def test_reproducible_and_distinct():
    a = testgen.su3_field(1000, seed=1710, field_id=0)
    b = testgen.su3_field(1000, seed=1710, field_id=0)
    c = testgen.su3_field(1000, seed=1710, field_id=1)
    d = testgen.su3_field(1000, seed=1711, field_id=0)
    assert testgen.buffer_sha256(a) == testgen.buffer_sha256(b)
    assert not np.array_equal(a, c) and not np.array_equal(a, d)


def test_site_independent_of_volume_and_chunking():
    full = testgen.su3_field(500, field_id=3)
    part = testgen.su3_field(100, field_id=3, s_begin=250)
    assert np.array_equal(full[250:350], part)
    sites = [0, 17, 499, 250]
    assert np.array_equal(testgen.su3_sites(sites, field_id=3), full[sites])


def test_every_matrix_in_su3():
    u = to_complex(testgen.su3_field(20000, field_id=4))
    uud = np.matmul(u, np.conj(np.transpose(u, (0, 2, 1))))
    assert np.max(np.abs(uud - np.eye(3))) <= 4e-15  # ~18 ulp: generation + this check
    assert np.max(np.abs(np.linalg.det(u) - 1.0)) <= 4e-15


def test_haar_moments():
    """Haar measure on SU(3): E|u_ij|^2 = 1/3, Var|u_ij|^2 = 1/12 - 1/9
    ... checked through the mean only (5 sigma), and E u_ij = 0."""
    n = 50000
    u = to_complex(testgen.su3_field(n, field_id=5))
    p = np.abs(u) ** 2
    # for Haar U(N)/SU(N), |u_ij|^2 ~ Beta(1, N-1): var = (N-1)/(N^2 (N+1))
    sigma = np.sqrt(2.0 / (9.0 * 4.0) / n)
    assert np.all(np.abs(p.mean(axis=0) - 1.0 / 3.0) < 5 * sigma)
    assert np.all(np.abs(u.mean(axis=0)) < 5 * np.sqrt(1.0 / 3.0 / n))


def test_raw_stream_known_values():
    """SplitMix64 finaliser on the counter stream: the first draw of
    (seed=0, field 0) recomputed with Python integers."""
    M = (1 << 64) - 1

    def mix(z):
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        return z ^ (z >> 31)

    for seed, fid, n in ((0, 0, 0), (1710, 100, 5), (2 ** 63, 7, 123456789)):
        key = mix(seed ^ mix(fid + 1))
        assert testgen.u64(seed, fid, n) == mix((key + (n + 1) * 0x9E3779B97F4A7C15) & M)


def test_batch_list():
    lat = testgen.batch_lattices(64)
    assert len(lat) == 64
    assert {d for d, _ in lat} <= set(testgen.BATCH_VOLUMES)
    assert any(c for _, c in lat) and not all(c for _, c in lat)
    assert lat == testgen.batch_lattices(64)
