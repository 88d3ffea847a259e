"""A small baseline-JPEG writer for crafted test inputs (test infrastructure).

It writes a file from symbol level up, so tests can build streams that a
normal encoder never emits: coefficient values at the limits of the baseline
format, invalid (run, size) symbols, zero runs past the last coefficient.
Markers and entropy coding follow ITU-T T.81 (B.2 syntax, Annex C code
assignment, F.1.2 coding of DC differences and AC run/size symbols, byte
stuffing after 0xFF).  Neither the oracle nor the library uses this module.
"""
from __future__ import annotations

import numpy as np

# zigzag scan position -> natural index (T.81 Figure A.6)
ZIGZAG = [0, 1, 8, 16, 9, 2, 3, 10, 17, 24, 32, 25, 18, 11, 4, 5, 12, 19, 26, 33, 40, 48, 41, 34, 27,
          20, 13, 6, 7, 14, 21, 28, 35, 42, 49, 56, 57, 50, 43, 36, 29, 22, 15, 23, 30, 37, 44, 51, 58,
          59, 52, 45, 38, 31, 39, 46, 53, 60, 61, 54, 47, 55, 62, 63]


def flat_table(symbols, length):
    """BITS / HUFFVAL of a table giving every symbol a code of `length` bits."""
    assert len(symbols) < (1 << length)
    bits = [0] * 16
    bits[length - 1] = len(symbols)
    return bits, list(symbols)


DC_SYMBOLS = list(range(12))
AC_SYMBOLS = [0x00, 0xF0] + [(r << 4) | s for r in range(16) for s in range(1, 11)]


def default_tables(extra_ac=()):
    """DC tables of all 12 categories (4-bit codes) and AC tables of the 162
    baseline symbols plus `extra_ac` (8-bit codes)."""
    dc = flat_table(DC_SYMBOLS, 4)
    ac = flat_table(AC_SYMBOLS + list(extra_ac), 8)
    return {"dc0": dc, "ac0": ac, "dc1": dc, "ac1": ac}


def _codes(bits, vals):
    """Annex C: code of each symbol."""
    out, code, k = {}, 0, 0
    for l in range(1, 17):
        for _ in range(bits[l - 1]):
            out[vals[k]] = (code, l)
            code += 1
            k += 1
        code <<= 1
    return out


class _Bits:
    def __init__(self):
        self.out = bytearray()
        self.acc = 0
        self.n = 0

    def put(self, v, n):
        for i in range(n - 1, -1, -1):
            self.acc = (self.acc << 1) | ((v >> i) & 1)
            self.n += 1
            if self.n == 8:
                self.out.append(self.acc)
                if self.acc == 0xFF:
                    self.out.append(0)
                self.acc, self.n = 0, 0

    def flush(self):
        while self.n:
            self.put(1, 1)


def _size(v):
    a, s = abs(int(v)), 0
    while a:
        s += 1
        a >>= 1
    return s


def _bits_of(v, s):
    """The s appended bits of value v (F.1.2.1: negative values as v - 1)."""
    return (v if v >= 0 else v + (1 << s) - 1) & ((1 << s) - 1)


def du_symbols(zz):
    """AC symbols of one data unit's coefficients in zigzag order: a list of
    (run/size byte, value) ending with EOB unless coefficient 63 is set."""
    out, run = [], 0
    last = max([k for k in range(1, 64) if zz[k] != 0], default=0)
    for k in range(1, last + 1):
        if zz[k] == 0:
            run += 1
            continue
        while run > 15:
            out.append((0xF0, 0))
            run -= 16
        out.append(((run << 4) | _size(zz[k]), int(zz[k])))
        run = 0
    if last < 63:
        out.append((0x00, 0))
    return out


def mcus_from_coefs(coef, sampling):
    """coef: [n_mcu, n_du, 64] quantised coefficients in natural order ->
    per MCU, per data unit, (DC difference, AC symbols)."""
    n_du = 6 if sampling == 420 else 3
    pred = [0, 0, 0]
    mcus = []
    for m in range(coef.shape[0]):
        dus = []
        for d in range(n_du):
            c = (0 if d < 4 else d - 3) if sampling == 420 else d
            zz = [int(coef[m, d, ZIGZAG[k]]) for k in range(64)]
            dus.append((zz[0] - pred[c], du_symbols(zz)))
            pred[c] = zz[0]
        mcus.append(dus)
    return mcus


def write_jpeg(width, height, sampling, q_luma, q_chroma, mcus, tables=None):
    """Baseline JPEG bytes.  q_luma / q_chroma: 64 quantiser values in
    natural order (8-bit).  mcus: per MCU a list of data units, each
    (DC difference, [(run/size byte, value), ...]); the value of a symbol
    with size s is written in s appended bits."""
    tables = tables or default_tables()
    b = bytearray(b"\xFF\xD8")

    def seg(marker, payload):
        b.extend(bytes([0xFF, marker]) + (len(payload) + 2).to_bytes(2, "big") + bytes(payload))

    dqt = bytearray()
    for t, q in enumerate((q_luma, q_chroma)):
        dqt.append(t)
        dqt.extend(int(q[ZIGZAG[k]]) for k in range(64))
    seg(0xDB, dqt)
    hv = 0x22 if sampling == 420 else 0x11
    seg(0xC0, [8] + list(height.to_bytes(2, "big")) + list(width.to_bytes(2, "big")) +
        [3, 1, hv, 0, 2, 0x11, 1, 3, 0x11, 1])
    dht = bytearray()
    for cls_id, key in ((0x00, "dc0"), (0x10, "ac0"), (0x01, "dc1"), (0x11, "ac1")):
        bits, vals = tables[key]
        dht.append(cls_id)
        dht.extend(bits)
        dht.extend(vals)
    seg(0xC4, dht)
    seg(0xDA, [3, 1, 0x00, 2, 0x11, 3, 0x11, 0, 63, 0])
    codes = {k: _codes(*v) for k, v in tables.items()}
    w = _Bits()
    for dus in mcus:
        for d, (dc_diff, acs) in enumerate(dus):
            c = (0 if d < 4 else d - 3) if sampling == 420 else d
            dc, ac = codes["dc1" if c else "dc0"], codes["ac1" if c else "ac0"]
            s = _size(dc_diff)
            w.put(*dc[s])
            w.put(_bits_of(dc_diff, s), s)
            for rs, v in acs:
                w.put(*ac[rs])
                s = rs & 15
                w.put(_bits_of(v, s), s)
    w.flush()
    b.extend(w.out)
    b.extend(b"\xFF\xD9")
    return bytes(b)


def mcu_count(width, height, sampling):
    ms = 16 if sampling == 420 else 8
    return ((width + ms - 1) // ms) * ((height + ms - 1) // ms)


def random_coefs(rng, n_mcu, sampling, dc_max=2047, ac_max=1023, density=0.5):
    """Random quantised coefficients at the limits of the baseline format:
    ACs uniform in [-ac_max, ac_max] (a `density` share non-zero), DCs a
    random walk per component inside [-dc_max, dc_max] whose steps fit the
    11-bit DC difference categories."""
    n_du = 6 if sampling == 420 else 3
    coef = rng.integers(-ac_max, ac_max + 1, (n_mcu, n_du, 64))
    coef *= rng.random((n_mcu, n_du, 64)) < density
    pred = [0, 0, 0]
    for m in range(n_mcu):
        for d in range(n_du):
            c = (0 if d < 4 else d - 3) if sampling == 420 else d
            lo, hi = max(-dc_max, pred[c] - 2047), min(dc_max, pred[c] + 2047)
            pred[c] = int(rng.integers(lo, hi + 1))
            coef[m, d, 0] = pred[c]
    return coef.astype(np.int16)
