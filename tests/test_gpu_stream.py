"""exx_stream_rates through the C ABI: four finite positive rates and a
description of the winning launch shapes; argument errors come back as
EXX_EINVAL before anything is allocated."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1911_10630_amd import exx as X  # noqa: E402


def test_stream_rates_small_arrays():
    r = X.stream_rates(0, bytes_per_array=64 << 20, reps=1)
    for k in ("read", "copy", "triad", "cg"):
        assert np.isfinite(r[k]) and r[k] > 0.0, (k, r)
    assert "read" in r["detail"] and "cg" in r["detail"]


def test_stream_rates_rejects_bad_arguments():
    L = X.load()
    out = np.zeros(4)
    ptr = out.ctypes.data_as(C.c_void_p)
    assert L.exx_stream_rates(0, 1 << 19, 1, ptr, None, 0) == X.EXX_EINVAL     # under 1 MiB
    assert L.exx_stream_rates(0, 64 << 20, 0, ptr, None, 0) == X.EXX_EINVAL    # no timed launch
    assert L.exx_stream_rates(0, 64 << 20, 1, None, None, 0) == X.EXX_EINVAL   # no output
