"""The counting kernel's integer scheme, modelled on the CPU with the
documented semantics of the gfx9 instructions it uses, against a direct count
of the Heaviside predicate n.s > D' (Sec. 2 estimator).

Per (sample, integrand pair) the kernel forms r = n.s - D' - 1, packs the two
residues' sign bits as 0x00/0xFF bytes into the two 16-bit halves of a word
(v_perm_b32 selectors 9 and 11), sums words with 32-bit adds, turns each half
(255 x misses) into misses with (x + 255) >> 8, adds the lanes of an item and
subtracts from N.  The model checks that no half ever carries into the other
at the kernel's limits (64 samples per lane, N <= 4096) and that the counts
equal the direct ones, including all-hit and all-miss rows."""
import numpy as np
import pytest

M32 = 0xFFFFFFFF


def v_perm_b32(s0, s1, sel):
    """Byte permute of the 64-bit value {s0, s1} (s1 in bits 31:0): selector
    bytes 0-7 pick a byte, 8-11 repeat bit 15, 31, 47 or 63 over the byte,
    12 gives 0x00 and 13-15 give 0xFF."""
    data = ((s0 & M32) << 32) | (s1 & M32)
    out = 0
    for i in range(4):
        b = (sel >> (8 * i)) & 0xFF
        if b < 8:
            v = (data >> (8 * b)) & 0xFF
        elif b < 12:
            v = 0xFF if (data >> (16 * (b - 8) + 15)) & 1 else 0
        elif b == 12:
            v = 0
        else:
            v = 0xFF
        out |= v << (8 * i)
    return out


def halves_div255(x):
    lo, hi = x & 0xFFFF, x >> 16
    return (((lo + 255) & 0xFFFF) >> 8) | ((((hi + 255) & 0xFFFF) >> 8) << 16)


def kernel_counts(nrm, thr, samples):
    """Counts of two integrands (normals nrm[2] as int16 pairs, thresholds
    thr[2]) over samples [N][2] (centred int16), the way the kernel's lanes
    split them: min(N, 64) samples per lane, N / 64 lanes per item."""
    n = len(samples)
    ns = min(n, 64)
    lanes = n // ns
    total = 0
    for lane in range(lanes):
        a = 0
        for s in samples[lane * ns:(lane + 1) * ns]:
            r0 = int(nrm[0][0]) * int(s[0]) + int(nrm[0][1]) * int(s[1]) - thr[0] - 1
            r1 = int(nrm[1][0]) * int(s[0]) + int(nrm[1][1]) * int(s[1]) - thr[1] - 1
            assert abs(r0) < 2 ** 31 and abs(r1) < 2 ** 31
            a = (a + v_perm_b32(r1 & M32, r0 & M32, 0x0C0B0C09)) & M32
            assert (a & 0xFFFF) <= 255 * 64 and (a >> 16) <= 255 * 64
        total = (total + halves_div255(a)) & M32
        assert (total & 0xFFFF) <= n and (total >> 16) <= n
    c = ((n | (n << 16)) - total) & M32
    return c & 0xFFFF, c >> 16


def direct_counts(nrm, thr, samples):
    s = samples.astype(np.int64)
    return tuple(int(np.sum(s @ np.asarray(nrm[i], np.int64) > thr[i])) for i in range(2))


def test_perm_selectors_give_sign_bytes():
    for hi in (-1, 0, 5, -(2 ** 30), 2 ** 30):
        for lo in (-7, 0, 3, -(2 ** 30), 2 ** 30):
            w = v_perm_b32(hi & M32, lo & M32, 0x0C0B0C09)
            assert w == (0xFF if lo < 0 else 0) | ((0xFF if hi < 0 else 0) << 16)


def test_halves_division_is_exact():
    for m in range(256):
        assert halves_div255(255 * m | (255 * (255 - m)) << 16) == m | (255 - m) << 16


@pytest.mark.parametrize("n", [1, 2, 4, 16, 64, 128, 256, 1024, 4096])
def test_counts_equal_direct_predicate(n):
    rng = np.random.default_rng(n)
    samples = rng.integers(-2 ** 15, 2 ** 15, size=(n, 2))
    for trial in range(4):
        nrm = rng.integers(-2 ** 14, 2 ** 14, size=(2, 2))
        thr = [int(rng.integers(-2 ** 30, 2 ** 30)) for _ in range(2)]
        if trial == 1:       # every sample misses the first, hits the second
            thr = [2 ** 30, -2 ** 30 - 1]
        if trial == 2:       # padded integrand: normal (0, 0), threshold 0
            nrm[0] = 0
            thr[0] = 0
        assert kernel_counts(nrm, thr, samples) == direct_counts(nrm, thr, samples)
