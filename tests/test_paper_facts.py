"""The paper's printed grid counts and sizes fix how its ranges are read:
half-open (upper end excluded) and complex single precision storage."""
import json
import os

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")))


def _half_open(lo, hi, step):
    return len(range(lo, hi, step))


def test_experiment1_entry_count_is_half_open():
    g = GOLD["experiment1_grid"]
    n = _half_open(*g["t1"]) * _half_open(*g["t2"]) * _half_open(*g["df"])
    assert n == g["entries"]
    closed = (_half_open(*g["t1"]) + 1) * (_half_open(*g["t2"]) + 1) * (_half_open(*g["df"]) + 1)
    assert closed != g["entries"]


def test_experiment2_size_is_complex64():
    g = GOLD["experiment2_grid"]
    n = _half_open(*g["t1"]) * _half_open(*g["t2"]) * _half_open(*g["df"])
    gib = n * g["timepoints"] * 8 / 2 ** 30
    assert round(gib, 1) == g["gigabytes"]


def test_experiment2_speedups_consistent():
    s = GOLD["experiment2_speedups"]
    assert round(s["brute_s"] / s["nodict_s"]) == s["nodict_x"]
    assert abs(s["brute_s"] / s["fulldict_s"] - s["fulldict_x"]) < 1
    assert abs(s["brute_s"] / s["dfdict_s"] - s["dfdict_x"]) < 1
