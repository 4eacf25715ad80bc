"""The oracle pinned to brute force, closed forms, invariants and the paper's
printed example and sizes (CPU only)."""
import pytest

import oracle
import pins
from paper_2210_01465_amd import synth


@pytest.fixture(scope="module")
def lib():
    oracle.load()
    return oracle.LIB


@pytest.mark.parametrize("check", pins.QUICK, ids=lambda c: c.__name__)
def test_quick_pin(lib, check):
    check(lib)


def test_mid_grid_degrees_and_dag(lib):
    s = synth.mid()
    pins.check_grid_degrees(lib, [s])
    pins.check_dag_identity(lib, [s], nbs=("hamming", "adjacent"))
    pins.check_invariants(lib, [s])


def test_tiny_invariants(lib):
    spaces = [synth.tiny(seed) for seed in range(10)]
    pins.check_grid_degrees(lib, spaces)
    pins.check_dag_identity(lib, spaces, nbs=("hamming", "adjacent"))
    pins.check_invariants(lib, spaces)


@pytest.mark.slow
def test_large_grid_degrees_and_dag(lib):
    s = synth.large()
    pins.check_grid_degrees(lib, [s], nbs=("hamming",))
    pins.check_dag_identity(lib, [s])
