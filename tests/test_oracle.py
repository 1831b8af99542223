"""The CPU oracle against its pins (no GPU)."""
import os
import tempfile

import pytest

import oracle
from tests import oracle_pins as pins


@pytest.fixture(scope="module")
def orc():
    return oracle.default()


def test_hand_cases(orc):
    pins.pin_hand_cases(orc)


def test_exhaustive_binary(orc):
    pins.pin_exhaustive_binary(orc, nmax=9)


def test_binary_total_closed_form(orc):
    pins.pin_binary_total_closed_form(orc, n=12)


def test_random_vs_library(orc):
    pins.pin_random_vs_library(orc, cases=100000)


def test_closed_forms(orc):
    pins.pin_closed_forms(orc)


def test_planted_and_edges(orc):
    pins.pin_planted_and_edges(orc)


def test_statistics(orc):
    pins.pin_statistics(orc)


def test_empty_pattern_rejected(orc):
    with pytest.raises(ValueError):
        orc.find_all(b"abc", b"")


@pytest.mark.parametrize("mutant", [1, 2, 3, 4, 5])
def test_planted_mistakes_are_caught(mutant):
    """Each numbered mistake planted into the oracle source fails at least one pin."""
    with tempfile.TemporaryDirectory() as d:
        so = oracle.build(os.path.join(d, "liboracle_m%d.so" % mutant), mutant=mutant)
        bad = pins.failing_pins(oracle.Oracle(so))
    assert bad, "mutant %d survived every pin" % mutant
