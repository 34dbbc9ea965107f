"""The sampler's counter-based generator (Philox4x32-10) against its published known-answer vectors."""
import numpy as np
import pytest


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds, written from the definition by Salmon et al. (SC 2011)."""
    x, y, z, w = ctr
    k0, k1 = key
    m = 0xFFFFFFFF
    for _ in range(10):
        p0 = 0xD2511F53 * x
        p1 = 0xCD9E8D57 * z
        x, y, z, w = ((p1 >> 32) ^ y ^ k0) & m, p1 & m, ((p0 >> 32) ^ w ^ k1) & m, p0 & m
        k0 = (k0 + 0x9E3779B9) & m
        k1 = (k1 + 0xBB67AE85) & m
    return (x, y, z, w)


# known-answer vectors distributed with the Random123 library for philox4x32_10
KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF), (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,expect", KAT)
def test_philox_known_answers(ctr, key, expect):
    assert philox4x32_10(ctr, key) == expect


@pytest.mark.gpu
def test_device_philox_matches_reference():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_06300_amd as lps
    seed, first, n = 0x1234_5678_9ABC_DEF0, (1 << 33) - 5, 257
    got = lps.philox4x32_10(seed, first, n).cpu().numpy()
    for i in range(n):
        c = first + i
        ref = philox4x32_10((c & 0xFFFFFFFF, c >> 32, 0, 0), (seed & 0xFFFFFFFF, seed >> 32))
        assert tuple(int(v) for v in got[i]) == ref
