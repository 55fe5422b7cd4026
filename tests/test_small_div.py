"""Exhaustive check of the spreading kernel's small integer division,
floor(a / b) = (int)(fl(a * r) + 1e-3) for 0 <= a < 128 and 1 <= b <= 128,
where r is the hardware single-precision reciprocal of b.  The GPU's
reciprocal is accurate to 1 ulp; the check lets r be anywhere within 2 ulp of
1/b and rounds the product and the bias in single precision, as the device
does.  (The division itself runs on the GPU in every spreading test.)"""
import numpy as np


def test_small_div_is_exact_for_every_operand_pair():
    a = np.arange(128, dtype=np.float32)
    bias = np.float32(1.0e-3)
    for b in range(1, 129):
        r0 = np.float32(1.0) / np.float32(b)
        want = np.arange(128) // b
        for ulps in range(-2, 3):
            r = r0
            for _ in range(abs(ulps)):
                r = np.nextafter(r, np.float32(np.inf) if ulps > 0 else np.float32(0))
            prod = (a * r).astype(np.float32)
            got = np.floor((prod + bias).astype(np.float32)).astype(np.int64)
            assert np.array_equal(got, want), (b, ulps)
