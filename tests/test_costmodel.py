"""The Table 1 cost model against independently computed values."""
import pytest

from paper_2403_06218_amd import costmodel


@pytest.mark.parametrize("b,q,r,expected", [
    (32, 512, 512, "5.536e8"),
    (256, 4096, 4096, "2.834e11"),
    (256, 16384, 16384, "1.773e13"),
    (64, 32768, 32768, "1.4088e14"),
    (128, 32768, 32768, "1.4101e14"),
    (256, 32768, 32768, "1.4129e14"),
    (256, 65536, 65536, "1.128e15"),
    (16, 1000000, 64, "1.79e10"),
])
def test_ca3_values(b, q, r, expected):
    """Reference values evaluated separately from Table 1's expressions, printed
    to 3-5 significant digits: agreement to half a unit of the last digit."""
    mant, exp = expected.split("e")
    decimals = len(mant.split(".")[1])
    half_ulp = 0.5 * 10.0 ** (int(exp) - decimals)
    assert abs(costmodel.ca3(b, q, r) - float(expected)) <= half_ulp


def test_ca3_leading_term_and_pieces():
    # CA3 -> 4 q r^2 as b / r -> 0; one block is exactly CA4.
    q = r = 1 << 15
    assert abs(costmodel.ca3(64, q, r) / (4.0 * q * r * r) - 1) < 0.02
    assert costmodel.ca3(128, 1000, 128) == costmodel.ca4(128, 1000)
    assert costmodel.ca3(128, 1000, 256) == costmodel.ca4(128, 1000) + costmodel.ca5(128, 1000, 128)
    # Brute-force count of the two block projections + updates of Alg. 5 (S1, S2, S6, S7):
    b, q, s = 3, 7, 5
    count = 0
    for _pass in range(2):
        count += 2 * s * b * q      # H = P^T Q: s*b dot products of length q
        count += 2 * q * b * s      # Q -= P H: q*b dot products of length s
    assert count == 8 * b * q * s
