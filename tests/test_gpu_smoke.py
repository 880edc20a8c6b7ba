"""`__graft_entry__.smoke()` (one small assignment on the GPU, checked against the oracle) runs
under the test suite too."""
import pytest

pytestmark = pytest.mark.gpu


def test_smoke():
    import __graft_entry__ as entry
    entry.smoke()
