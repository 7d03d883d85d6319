"""Host-side logic of the autotuner: the Lemma 3.2 bound it filters Z with,
the choice of the fastest candidate and the stored table (no GPU needed)."""
import math

from paper_2008_01765_amd import autotune


def test_log2_eps_matches_lemma_3_2_values():
    # log2 of B log2 B e^(-Z/6) at n = 2^28 (B = 2n/Z): the worked values of
    # the bound at the headline size
    for z, want in ((256, -36.2), (512, -98.8), (1024, -223.0)):
        assert abs(autotune.log2_eps(1 << 28, z) - want) < 0.1
    # single bin: no level, no overflow
    assert autotune.log2_eps(100, 512) == -math.inf


def test_log2_eps_closed_form():
    for n, z in ((1 << 16, 512), (1 << 24, 512), (12345, 1024), (1 << 20, 256)):
        B = 1
        while B * z < 2 * n:
            B *= 2
        L = int(math.log2(B))
        want = math.log2(B * L * math.exp(-z / 6.0))
        assert abs(autotune.log2_eps(n, z) - want) < 1e-9


def test_admissible_z_at_80_bits():
    assert autotune.admissible_z(1 << 28, 80) == [512, 1024]
    assert autotune.admissible_z(1 << 28, 30) == [256, 512, 1024]
    assert autotune.admissible_z(1 << 10, 80) == [512, 1024]


def test_best_picks_fastest_first_on_ties():
    assert autotune.best([((512, 4), 3.0), ((512, 3), 2.0), ((1024, 4), 2.5)]) == (512, 3)
    assert autotune.best([("a", 1.0), ("b", 1.0)]) == "a"


def test_table_round_trip(tmp_path):
    tab = [{"rec": 8, "log2n": 20, "z": 512, "k": 4, "tile": 2048, "ns_per_record": 0.1, "instances": 4}]
    p = tmp_path / "t.json"
    autotune.save(tab, str(p), "gpu")
    assert autotune.load(str(p)) == tab


def test_tile_candidates_fit_lds():
    # 16384 records of 16 bytes would need 256 KiB of LDS per workgroup
    assert autotune.tile_candidates(8) == (1024, 2048, 4096, 8192, 16384)
    assert autotune.tile_candidates(16) == (1024, 2048, 4096, 8192)
