import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    from oracle import build as obuild
    if not os.path.exists(oracle.LIB_PATH):
        obuild.build()
    return oracle


def load_table1():
    vals = {}
    with open(os.path.join(ROOT, "tests", "golden", "table1.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split()
            vals[k] = float(v)
    return vals


U32 = 2.0 ** -24  # unit roundoff of FP32


def fp32_errors(got, ref, fields):
    """Per-field FP32-path error against an FP64 reference, two ways:
    ||d|| / ||f|| and ||d|| / ||f - fbar(z)||, fbar the horizontal mean per
    level (the second does not hide an error behind a large mean such as
    theta_l ~ 290 K)."""
    out = {}
    for k in fields:
        a, b = got[k], ref[k]
        d = np.linalg.norm(a - b)
        nb = np.linalg.norm(b)
        na = np.linalg.norm(b - b.mean(axis=(1, 2), keepdims=True))
        out[k] = (d / (nb if nb > 0 else 1.0), d / (na if na > 0 else 1.0), nb / max(na, 1e-300))
    return out


def assert_fp32(errs, bar=1e-5, ulps=64):
    """Bars of the FP32 path, per field and step: relative L2 <= bar, and
    relative to the field's horizontal anomaly <= max(bar, ulps u32 ||f|| /
    ||f - fbar||).  The second term is the floor set by storage alone: one
    FP32 rounding of every value already moves a field by ~u32 ||f|| / sqrt(3),
    and a step rounds each value through a few tens of operations; so the
    anomaly bar binds wherever the anomaly is large enough for FP32 to
    resolve it to 1e-5, and reduces to 64 roundings of the field otherwise."""
    for k, (e, ea, ratio) in errs.items():
        assert e <= bar, (k, "relative L2", e)
        assert ea <= max(bar, ulps * U32 * ratio), (k, "relative to anomaly", ea, ratio)


def fmt_fp32(errs):
    return " ".join(f"{k} {e:.2e}/{ea:.2e}" for k, (e, ea, _) in errs.items())
