"""Constant tables compiled into the HIP kernels, checked against their definitions."""
import math
import os
import re
from decimal import Decimal, getcontext

HERE = os.path.dirname(os.path.abspath(__file__))
DEVICE_H = os.path.join(HERE, "..", "paper_2102_09811_amd", "csrc", "hb_device.h")


def test_exp2_table_is_correctly_rounded():
    """kExp2Tab[j] must be 2^{-j/64} rounded to the nearest double (the table-based e^{-w})."""
    src = open(DEVICE_H).read()
    body = re.search(r"kExp2Tab\[64\]\s*=\s*\{([^}]*)\}", src).group(1)
    vals = [float.fromhex(t) for t in re.findall(r"0x[0-9a-fA-F.]+p[+-]\d+", body)]
    assert len(vals) == 64
    getcontext().prec = 60
    for j, v in enumerate(vals):
        exact = Decimal(2) ** (Decimal(-j) / 64)
        assert v == float(exact), j
        # and no neighbouring double is closer
        err = abs(Decimal(v) - exact)
        assert err <= abs(Decimal(math.nextafter(v, 0.0)) - exact)
        assert err <= abs(Decimal(math.nextafter(v, 2.0)) - exact)


def test_exp2_table256_is_correctly_rounded():
    """kExp2Tab256[j] must be 2^{-j/256} rounded to the nearest double (the table of exp_neg_m)."""
    src = open(DEVICE_H).read()
    body = re.search(r"kExp2Tab256\[kExpTabN\]\s*=\s*\{([^}]*)\}", src).group(1)
    assert re.search(r"constexpr int kExpTabN = 256;", src)
    vals = [float.fromhex(t) for t in re.findall(r"0x[0-9a-fA-F.]+p[+-]\d+", body)]
    assert len(vals) == 256
    getcontext().prec = 60
    for j, v in enumerate(vals):
        exact = Decimal(2) ** (Decimal(-j) / 256)
        assert v == float(exact), j
        err = abs(Decimal(v) - exact)
        assert err <= abs(Decimal(math.nextafter(v, 0.0)) - exact)
        assert err <= abs(Decimal(math.nextafter(v, 2.0)) - exact)
