"""Host-side behaviour of the Python binding (no GPU)."""
import warnings

import pytest


def test_bf16_on_large_grids_warns():
    from paper_1903_12227_amd import api
    with pytest.warns(RuntimeWarning, match="FP16"):
        api._warn_bf16_large(api.Options(prec=api.MIX_BF16), 2048)
    with warnings.catch_warnings():
        warnings.simplefilter("error")
        api._warn_bf16_large(api.Options(prec=api.MIX_BF16), 512)
        api._warn_bf16_large(api.Options(prec=api.MIX_FP16), 2048)
        api._warn_bf16_large(api.Options(prec=api.FP64), 4096)
