"""Crafted baseline streams at and past the limits of T.81 (CPU only).

The oracle's sequential decoder and the library's index builder must agree
on what a baseline stream is: coefficients at the extremes of their
categories round-trip, and the invalid forms are rejected by both -- a
(run, size 0) symbol other than EOB (0/0) and ZRL (15/0), an AC size above
10 bits (T.81 F.1.2.2: baseline AC magnitudes take at most 10 bits), a run
of zeros past coefficient 63.  A quantised DC outside 12 bits in any data
unit is valid T.81 but outside the index format (JPT_E_RANGE)."""
import numpy as np
import pytest

import oracle
from paper_2510_08166_amd import jpt

from jpeg_writer import (default_tables, mcu_count, mcus_from_coefs, random_coefs, write_jpeg)

Q1 = np.ones(64, np.int64)


def oracle_decode(data):
    j = oracle.Jpeg(data)
    return j.decode()[0]


def one_mcu(acs, dc=0, sampling=444, tables=None):
    """A 8x8 (4:4:4) or 16x16 (4:2:0) image of one MCU: the luma data unit
    carries `acs`, the others are empty."""
    n_du = 6 if sampling == 420 else 3
    dus = [(dc, list(acs))] + [(0, [(0x00, 0)]) for _ in range(n_du - 1)]
    side = 16 if sampling == 420 else 8
    return write_jpeg(side, side, sampling, Q1, Q1, [dus], tables)


@pytest.mark.parametrize("sampling", [420, 444])
def test_extreme_coefficients_round_trip(sampling):
    """Every category at its largest magnitude: the decoded coefficients are
    the written ones (EXTEND, F.2.2.1, at sizes 1..11), and the library's
    spliced stream decodes to them MCU by MCU."""
    rng = np.random.default_rng(5)
    w, h = 40, 24
    coef = random_coefs(rng, mcu_count(w, h, sampling), sampling)
    coef[0, 0, 1:11] = [(1 << s) - 1 if s % 2 else -((1 << s) - 1) for s in range(1, 11)]
    data = write_jpeg(w, h, sampling, np.full(64, 255), np.full(64, 255), mcus_from_coefs(coef, sampling))
    assert np.array_equal(oracle_decode(data), coef)
    li = jpt.build_index(data)
    j = oracle.Jpeg(data)
    for m in range(j.n_mcu):
        rc, out, end = j.decode_stripped_mcu(li.stream, li.info.stream_bits, li.records, m)
        assert rc == 0 and np.array_equal(out, coef[m])


def test_run_size_zero_other_than_eob_and_zrl_is_corrupt():
    tables = default_tables(extra_ac=[0x10])
    good = one_mcu([(0x01, 1), (0x00, 0)], tables=tables)
    assert oracle_decode(good)[0, 0, 1] == 1
    bad = one_mcu([(0x01, 1), (0x10, 0), (0x00, 0)], tables=tables)
    with pytest.raises(oracle.OracleError):
        oracle_decode(bad)
    with pytest.raises(jpt.JptError) as e:
        jpt.build_index(bad)
    assert e.value.status == jpt.JPT_E_CORRUPT


def test_ac_size_above_ten_is_corrupt():
    tables = default_tables(extra_ac=[0x0B])
    bad = one_mcu([(0x0B, 1500), (0x00, 0)], tables=tables)
    with pytest.raises(oracle.OracleError):
        oracle_decode(bad)
    with pytest.raises(jpt.JptError) as e:
        jpt.build_index(bad)
    assert e.value.status == jpt.JPT_E_CORRUPT


def test_zero_run_reaching_exactly_64_is_valid():
    """ZRL at positions 48..63 ends the data unit without EOB."""
    acs = [(0xF0, 0)] * 2 + [(0xE1, 1)] + [(0xF0, 0)]    # zeros 1..32, 33..46, 1 at 47, zeros 48..63
    c = oracle_decode(one_mcu(acs))
    zz = np.zeros(64, np.int64)
    zz[47] = 1
    assert np.array_equal(c[0, 0][oracle.ZIGZAG], zz)
    jpt.build_index(one_mcu(acs))


def test_zero_run_past_63_is_corrupt():
    acs = [(0xF0, 0)] * 2 + [(0xF1, 1)] + [(0xF0, 0)]    # 1 at 48, then a ZRL over 49..64
    with pytest.raises(oracle.OracleError):
        oracle_decode(one_mcu(acs))
    with pytest.raises(jpt.JptError) as e:
        jpt.build_index(one_mcu(acs))
    assert e.value.status == jpt.JPT_E_CORRUPT
    acs = [(0xF0, 0)] * 3 + [(0x21, 1)] + [(0xF0, 0)]    # 1 at 51, then a ZRL over 52..67
    with pytest.raises(oracle.OracleError):
        oracle_decode(one_mcu(acs))
    with pytest.raises(jpt.JptError):
        jpt.build_index(one_mcu(acs))


def test_dc_outside_12_bits_is_out_of_index_range():
    """Y1 of a 4:2:0 MCU at 2048 (Y0 at 2000, difference 48): the oracle
    decodes it, the index builder reports JPT_E_RANGE; at 2047 both accept."""
    for y1, ok in ((2047, True), (2048, False)):
        dus = [(2000, [(0x00, 0)]), (y1 - 2000, [(0x00, 0)])] + [(0, [(0x00, 0)])] * 4
        data = write_jpeg(16, 16, 420, Q1, Q1, [dus])
        c = oracle_decode(data)
        assert c[0, 1, 0] == y1
        if ok:
            jpt.build_index(data)
        else:
            with pytest.raises(jpt.JptError) as e:
                jpt.build_index(data)
            assert e.value.status == jpt.JPT_E_RANGE
