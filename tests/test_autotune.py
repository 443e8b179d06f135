"""The autotuner's choice rule (host logic, no GPU): a candidate replaces
the default only when its median time beats the default's by more than the
measured noise."""
from paper_1210_0748_amd import autotune


def test_keeps_default_within_noise():
    runs = {64: [1.00, 1.01, 0.99], 512: [0.985, 0.99, 0.98], 4096: [1.0, 1.02, 0.98]}
    choice, rep = autotune.choose(runs)
    assert choice == 4096 and rep["kept_default"] and rep["fastest"] == 512


def test_takes_clear_winner():
    runs = {64: [0.80, 0.81, 0.79], 512: [0.95, 0.96, 0.94], 4096: [1.0, 1.01, 0.99]}
    choice, rep = autotune.choose(runs)
    assert choice == 64 and not rep["kept_default"]


def test_noisy_default_needs_larger_gain():
    # the default's spread is 10%: a 12% gain is not enough (noise = 20%)
    runs = {512: [0.88, 0.88, 0.88], 4096: [1.0, 1.1, 0.9]}
    choice, rep = autotune.choose(runs)
    assert choice == 4096 and abs(rep["noise"] - 0.2) < 1e-9
    runs = {512: [0.7, 0.7, 0.7], 4096: [1.0, 1.1, 0.9]}
    assert autotune.choose(runs)[0] == 512
