"""The benchmark's FLOP model reproduces the paper's per-element FLOP table exactly."""
import json
import os

import bench

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_flops_table.json")


def test_flop_model_matches_paper_table():
    g = json.load(open(GOLD))
    for p, f, fd in zip(g["p"], g["flops_per_element"], g["flops_per_dof"]):
        assert bench.flops_per_element(p) == f
        assert round(bench.flops_per_element(p) / (3 * p ** 3)) == fd


def test_algorithmic_bytes():
    assert bench.algorithmic_bytes(100, 10, 8) == 16 * 100 + 96 * 10
    assert bench.algorithmic_bytes(100, 10, 4) == 8 * 100 + 48 * 10


def test_multi_gpu_request_exits():
    assert bench.main(["--gpus", "2"]) == 2
