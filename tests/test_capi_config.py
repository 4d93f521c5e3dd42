"""CPU tests of the kernel-variant thresholds of the C ABI (hs_config_set /
hs_config_get / hs_config_reset): no device is needed to read or set them."""

import pytest

from paper_1712_07297_amd import _lib as H

DEFAULTS = {
    "pivot_lds_max": 128,
    "trinv8_max": 128,
    "trinv12_max": 192,
    "qr_reg1_max": 64,
    "qr_reg2_max": 128,
    "wy_max": 128,
    "gram_splits_max": 256,
    "schur_ptab_max": 256,
    "schur_noff_max": 1024,
    "cholqr": 1,
    "crowded_min": 512,
    "gram_splits_crowded": 4,
    "wy_max_crowded": 0,
    "cholqr_crowded": 0,
    "dense_panel": 128,
    "apply_fwd": 0,
    "apply_wave": 1024,
    "apply_split_nrhs_max": 1,
    "compression": 0,
    "qrcp_below_eps": 1e-5,
}


def test_defaults_and_reset():
    H.config_reset()
    for k, v in DEFAULTS.items():
        assert H.config_get(k) == v, k
    try:
        H.config_set("dense_panel", 32)
        H.config_set("gram_splits_max", 1)
        assert H.config_get("dense_panel") == 32
        assert H.config_get("gram_splits_max") == 1
    finally:
        H.config_reset()
    assert H.config_get("dense_panel") == 128


@pytest.mark.parametrize("name,value", [("no_such_parameter", 1), ("pivot_lds_max", 129), ("pivot_lds_max", -1),
                                        ("dense_panel", 16.5), ("dense_panel", 8), ("gram_splits_max", 0),
                                        ("compression", 3), ("qrcp_below_eps", 2.0)])
def test_rejected_values_change_nothing(name, value):
    H.config_reset()
    with pytest.raises(H.HsError) as e:
        H.config_set(name, value)
    assert e.value.code == H.HS_ERR_ARG
    for k, v in DEFAULTS.items():
        assert H.config_get(k) == v
