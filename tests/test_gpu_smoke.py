"""The packaged smoke check (one small MTTKRP per precision, the FP8
preparation, two CP-ALS sweeps, all against the FP64 oracle) as a GPU test."""

import os
import sys

import pytest

pytestmark = pytest.mark.gpu


def test_smoke():
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import __graft_entry__
    __graft_entry__.smoke()
