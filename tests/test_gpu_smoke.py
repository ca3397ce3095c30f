"""The package's smoke check (one small A-apply in float32 and float64 and a
circulant PCG solve, each against the oracle) runs as a GPU test too, so the
test suite sees it fail as soon as the library's plan or results change."""

import os
import sys

import pytest

pytestmark = pytest.mark.gpu


def test_smoke_passes():
    from gpu_common import need_gpu
    need_gpu()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import __graft_entry__
    __graft_entry__.smoke()
