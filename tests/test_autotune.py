"""The autotuner's choice rule (host logic, no GPU): a candidate replaces
the default only when its median time beats the default's by more than the
measured noise. Candidates are single knobs or (medium_cap, radix_tile)
pairs."""
from paper_1210_0748_amd import autotune


def test_keeps_default_within_noise():
    runs = {64: [1.00, 1.01, 0.99], 512: [0.985, 0.99, 0.98], 4096: [1.0, 1.02, 0.98]}
    choice, rep = autotune.choose(runs, 4096)
    assert choice == 4096 and rep["kept_default"] and rep["fastest"] == 512


def test_takes_clear_winner():
    runs = {64: [0.80, 0.81, 0.79], 512: [0.95, 0.96, 0.94], 4096: [1.0, 1.01, 0.99]}
    choice, rep = autotune.choose(runs, 4096)
    assert choice == 64 and not rep["kept_default"]


def test_noisy_default_needs_larger_gain():
    # the default's spread is 10%: a 12% gain is not enough (noise = 20%)
    runs = {512: [0.88, 0.88, 0.88], 4096: [1.0, 1.1, 0.9]}
    choice, rep = autotune.choose(runs, 4096)
    assert choice == 4096 and abs(rep["noise"] - 0.2) < 1e-9
    runs = {512: [0.7, 0.7, 0.7], 4096: [1.0, 1.1, 0.9]}
    assert autotune.choose(runs, 4096)[0] == 512


def test_pairs_of_cap_and_tile():
    d = autotune.DEFAULT
    assert d in autotune.CANDIDATES and len(autotune.CANDIDATES) == len(autotune.CAPS) * len(autotune.TILES)
    runs = {c: [1.0, 1.01, 0.99] for c in autotune.CANDIDATES}
    runs[(1024, 2048)] = [0.97, 0.98, 0.97]  # within the 3% floor: the default stays
    choice, rep = autotune.choose(runs, d)
    assert choice == d and rep["fastest"] == (1024, 2048)
    runs[(1024, 2048)] = [0.90, 0.91, 0.90]
    assert autotune.choose(runs, d)[0] == (1024, 2048)


def test_cache_key_separates_candidate_sets_and_workloads():
    class G:
        def __init__(self, n, e):
            self.num_nodes, self.src = n, [0] * e
    small = [G(20_000, 160_000)] * 4
    big = [G(2_000_000, 16_000_000)] * 4
    full = autotune.CANDIDATES
    caps_only = tuple((c, autotune.DEFAULT[1]) for c in autotune.CAPS)
    keys = {autotune.cache_key("gfx950", small, 5, full), autotune.cache_key("gfx950", small, 5, caps_only),
            autotune.cache_key("gfx950", big, 5, full), autotune.cache_key("gfx950", small, 10, full),
            autotune.cache_key("gfx942", small, 5, full)}
    assert len(keys) == 5
    assert autotune.cache_key("gfx950", small, 5, full) == autotune.cache_key("gfx950", list(small), 5, list(full))
