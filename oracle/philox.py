"""Philox4x64-10 and the Gaussian transform used for Wigner sampling (oracle side).

TEST INFRASTRUCTURE: part of the oracle; never imported by the product path.

The paper draws, for every grid point and stream, two Gaussian numbers (Sec.
"Initial conditions generation", Eq. (sample)) but names no generator. The
reading used here: a counter-based generator so that any stream can be
re-drawn from (seed, cell, stream) alone.

Generator: Philox4x64 with 10 rounds, as published by Salmon, Moraes, Dror and
Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11). One round maps
counter words (x0, x1, x2, x3) with key (k0, k1) to
    (hi(M1*x2) ^ x1 ^ k0,  lo(M1*x2),  hi(M0*x0) ^ x3 ^ k1,  lo(M0*x0))
and the key is bumped by the Weyl constants between rounds.

Gaussian transform (Box-Muller, 1958), written so that it is a fixed sequence
of correctly rounded IEEE-754 double operations (+, -, *, /, sqrt, floor,
frexp) with no library transcendental, so an independent implementation that
performs the same operations in the same order reproduces it bit for bit:
  u      = (floor(x / 2^12) + 1/2) * 2^-52                       in (0, 1)
  ln u   : u = m 2^e with m in [sqrt(1/2), sqrt(2));  s = (m-1)/(m+1);
           ln m = 2 s * sum_{k=0..12} s^(2k)/(2k+1)   (Horner, highest k first,
           coefficient 1/(2k+1) formed by one division);  ln u = e*ln2 + ln m
  angle  : t = 4 u2, q = floor(t), f = t - q; if f > 1/2: f -= 1, q += 1;
           theta = f * (pi/2) in [-pi/4, pi/4]
  sin    : p = 1; for k = 10..1: p = 1 - (p*theta^2) * r_k;  sin = theta*p,
           r_k = 1/((2k)(2k+1)) rounded once to double
  cos    : p = 1; for k = 10..1: p = 1 - (p*theta^2) * c_k;  cos = p,
           c_k = 1/((2k-1)(2k)) rounded once to double
           (multiplications by the rounded reciprocals, not divisions)
           rotated by q quarter turns
  z1 = sqrt(-2 ln u1) cos(2 pi u2),  z2 = sqrt(-2 ln u1) sin(2 pi u2)
"""
import numpy as np

MASK64 = (1 << 64) - 1
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15
PHILOX_W1 = 0xBB67AE8584CAA73B
PHILOX_ROUNDS = 10

LN2 = 0.6931471805599453
HALF_PI = 1.5707963267948966
SQRT_HALF = 0.7071067811865476


def _mulhilo(a, b):
    """(hi, lo) 64-bit halves of the 128-bit product a*b for uint64 arrays."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.uint64(b)
    m32 = np.uint64(0xFFFFFFFF)
    s32 = np.uint64(32)
    a0, a1 = a & m32, a >> s32
    b0, b1 = b & m32, b >> s32
    p00 = a0 * b0
    p01 = a0 * b1
    p10 = a1 * b0
    p11 = a1 * b1
    mid = (p00 >> s32) + (p01 & m32) + (p10 & m32)
    hi = p11 + (p01 >> s32) + (p10 >> s32) + (mid >> s32)
    lo = a * b
    return hi, lo


def philox4x64(ctr, key):
    """Philox4x64-10 block function.

    ctr: (4, n) uint64 array of counter words; key: (k0, k1) Python ints.
    Returns a (4, n) uint64 array of output words.
    """
    x0, x1, x2, x3 = (np.array(c, dtype=np.uint64) for c in ctr)
    k0, k1 = int(key[0]) & MASK64, int(key[1]) & MASK64
    with np.errstate(over="ignore"):
        for rnd in range(PHILOX_ROUNDS):
            if rnd > 0:
                k0 = (k0 + PHILOX_W0) & MASK64
                k1 = (k1 + PHILOX_W1) & MASK64
            hi0, lo0 = _mulhilo(x0, PHILOX_M0)
            hi1, lo1 = _mulhilo(x2, PHILOX_M1)
            x0, x1, x2, x3 = (hi1 ^ x1 ^ np.uint64(k0), lo1,
                              hi0 ^ x3 ^ np.uint64(k1), lo0)
    return np.stack([x0, x1, x2, x3])


def uniform52(x):
    """Map uint64 words to doubles (floor(x/2^12) + 1/2) * 2^-52, strictly inside (0, 1)."""
    top = (np.asarray(x, dtype=np.uint64) >> np.uint64(12)).astype(np.float64)
    return (top + 0.5) * (2.0 ** -52)


def log_series(u):
    """Natural log of u in (0, 1] by binary exponent extraction and the atanh series."""
    u = np.asarray(u, dtype=np.float64)
    m, e = np.frexp(u)                     # u = m * 2^e, m in [1/2, 1)
    low = m < SQRT_HALF
    m = np.where(low, m * 2.0, m)
    e = np.where(low, e - 1, e).astype(np.float64)
    s = (m - 1.0) / (m + 1.0)
    t = s * s
    p = np.full_like(s, 1.0 / 25.0)
    for k in range(11, -1, -1):
        p = p * t + 1.0 / (2 * k + 1)
    lnm = (s + s) * p
    return e * LN2 + lnm


def cos_sin_turn(u):
    """(cos, sin) of 2*pi*u for u in (0, 1) via quarter-turn reduction and Taylor series."""
    u = np.asarray(u, dtype=np.float64)
    t4 = 4.0 * u
    q = np.floor(t4)
    f = t4 - q
    up = f > 0.5
    f = np.where(up, f - 1.0, f)
    q = np.where(up, q + 1.0, q)
    theta = f * HALF_PI
    th2 = theta * theta
    ps = np.ones_like(theta)
    pc = np.ones_like(theta)
    for k in range(10, 0, -1):
        # multiply by the correctly rounded reciprocal of the factorial ratio
        ps = 1.0 - (ps * th2) * (1.0 / float((2 * k) * (2 * k + 1)))
        pc = 1.0 - (pc * th2) * (1.0 / float((2 * k - 1) * (2 * k)))
    s = theta * ps
    c = pc
    quad = q.astype(np.int64) & 3
    cos_out = np.select([quad == 0, quad == 1, quad == 2], [c, -s, -c], s)
    sin_out = np.select([quad == 0, quad == 1, quad == 2], [s, c, -s], -c)
    return cos_out, sin_out


def box_muller(x0, x1):
    """Two independent N(0,1) doubles per pair of uint64 words."""
    u1 = uniform52(x0)
    u2 = uniform52(x1)
    r = np.sqrt(-2.0 * log_series(u1))
    c, s = cos_sin_turn(u2)
    return r * c, r * s
