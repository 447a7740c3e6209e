"""The round-trip smoke check (`__graft_entry__.smoke`): one small solve per
precision on cuda:0 against the oracle's direct solution."""

import os
import sys

import pytest

pytestmark = pytest.mark.gpu


def test_smoke_runs():
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import __graft_entry__
    __graft_entry__.smoke()
