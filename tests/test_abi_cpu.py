"""C ABI checks that need no GPU: the library loads, exports every symbol
include/salo.h declares, and host-side validation returns the documented
status codes without touching a device."""
import ctypes
import os
import re

import pytest

from paper_2301_09310_amd import salo

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "salo.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(salo_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(salo.LIB_PATH):
        pytest.fail("libsalo.so is not built (python -m paper_2301_09310_amd.build)")
    return salo.load()


def test_header_declares_the_boundary():
    names = _declared_functions()
    for n in ["salo_align_batch", "salo_align_batch_ex", "salo_reserve",
              "salo_error_count", "salo_last_timing", "salo_set_bins", "salo_get_bins",
              "salo_last_error", "salo_release", "salo_version", "salo_pack_bases",
              "salo_align_starts", "salo_align_batch_n", "salo_align_batch_banded",
              "salo_align_trace"]:
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_version(lib):
    assert lib.salo_version() == 1


SC = salo.Scoring(1, -4, 6, 1)
NULL = ctypes.c_void_p(0)
BUF = ctypes.create_string_buffer(64)
ADDR = ctypes.addressof(BUF)


def _call(n, sc=SC, ptr=ADDR, opts=None):
    o = opts if opts is not None else salo.make_options()
    return salo.load().salo_align_batch_ex(ptr, ptr, ptr, ptr, n, sc, ptr, ptr, ptr, NULL,
                                           ctypes.byref(o))


def test_zero_pairs_is_a_noop(lib):
    assert _call(0, ptr=None) == 0


def test_negative_count(lib):
    assert _call(-1) == -1
    assert "n_pairs" in lib.salo_last_error().decode()


@pytest.mark.parametrize("sc", [(0, -4, 6, 1), (1, 1, 6, 1), (1, -4, -1, 1), (1, -4, 6, -2),
                                (40000, -4, 6, 1), (1, -40000, 6, 1)])
def test_bad_scoring(lib, sc):
    assert _call(5, sc=salo.Scoring(*sc)) == -1


def test_null_pointer(lib):
    assert _call(5, ptr=None) == -1
    assert "NULL" in lib.salo_last_error().decode()


def test_misaligned_stream(lib):
    assert _call(5, ptr=ADDR + 1) == -1
    assert "aligned" in lib.salo_last_error().decode()


def test_bad_options(lib):
    o = salo.make_options()
    o.split_waves = 3
    assert _call(5, opts=o) == -1
    o = salo.make_options()
    o.no_f16 = 2
    assert _call(5, opts=o) == -1
    o = salo.make_options()
    o.mode = 9
    assert _call(5, opts=o) == -1


def test_too_many_pairs(lib):
    assert _call(1 << 31) == -1


def test_bin_table_roundtrip(lib):
    default = salo.get_bins()
    assert default[-1][0] == 65535 and len(default) >= 2
    table = [(100, 1, 1, 8), (1000, 1, 4, 32), (65535, 1, 16, 16), (65535, 0, 8, 16)]
    salo.set_bins(table)
    assert salo.get_bins() == table
    # three-field entries take 16 columns per lane
    salo.set_bins([(t[0], t[1], t[2]) for t in table])
    assert salo.get_bins() == [(t[0], t[1], t[2], 16) for t in table]
    salo.set_bins(None)
    assert salo.get_bins() == default


@pytest.mark.parametrize("table", [
    [(100, 1, 3), (65535, 1, 4), (65535, 0, 8)],          # lanes not a power of two
    [(100, 1, 1), (50, 1, 4), (65535, 1, 4), (65535, 0, 8)],  # m_hi decreasing
    [(100, 1, 1), (65535, 0, 8)],                          # 16-bit kind not closed
    [(65535, 1, 1)],                                       # no 32-bit kind
    [(100, 1, 1, 12), (65535, 1, 4), (65535, 0, 8)],      # columns not 8, 16 or 32
])
def test_bad_bin_tables(lib, table):
    before = salo.get_bins()
    with pytest.raises(salo.SaloError):
        salo.set_bins(table)
    assert salo.get_bins() == before


def _pack(n, chars=ADDR, off=ADDR, n_seqs=1, revcomp=0, packed=ADDR, inv=None, nmask=None):
    return salo.load().salo_pack_bases(chars, n, off, n_seqs, revcomp, packed, nmask, inv, NULL)


def test_pack_validation(lib):
    assert _pack(0, chars=None, off=None, packed=None) == 0       # no-op
    assert _pack(-1) == -1
    assert _pack(16, n_seqs=-1) == -1
    assert _pack(16, revcomp=2) == -1
    assert "revcomp" in lib.salo_last_error().decode()
    assert _pack(16, chars=None) == -1
    assert _pack(16, packed=None) == -1
    assert _pack(16, off=None, revcomp=1) == -1
    assert _pack(16, chars=ADDR + 1) == -1
    assert "aligned" in lib.salo_last_error().decode()
    assert _pack(16, packed=ADDR + 2) == -1
    assert _pack(16, off=ADDR + 4, revcomp=1) == -1
    assert _pack(16, inv=ADDR + 4) == -1
    assert _pack(16, nmask=ADDR + 2) == -1


def _starts(n, ptr=ADDR, ans=ADDR, opts=None, mask=None):
    o = opts if opts is not None else salo.make_options()
    return salo.load().salo_align_starts(ptr, mask, ptr, ptr, mask, ptr, n, SC, ans, ans, ans,
                                         ptr, ptr, NULL, ctypes.byref(o))


def test_starts_validation(lib):
    assert _starts(0, ptr=None, ans=None) == 0
    assert _starts(-1) == -1
    assert _starts(5, ans=None) == -1
    assert _starts(5, ans=ADDR + 2) == -1
    assert _starts(5, ptr=ADDR + 1) == -1
    assert _starts(5, mask=ADDR + 1) == -1
    o = salo.make_options(mode="plain")
    assert _starts(5, opts=o) == -5
    assert "persistent" in lib.salo_last_error().decode()


def test_masked_align_validation(lib):
    o = salo.make_options()
    f = salo.load().salo_align_batch_n
    assert f(None, None, None, None, None, None, 0, SC, None, None, None, NULL,
             ctypes.byref(o)) == 0
    assert f(ADDR, ADDR + 2, ADDR, ADDR, None, ADDR, 5, SC, ADDR, ADDR, ADDR, NULL,
             ctypes.byref(o)) == -1
    assert "mask" in lib.salo_last_error().decode()
    assert f(ADDR, None, ADDR, ADDR, None, ADDR, -1, SC, ADDR, ADDR, ADDR, NULL,
             ctypes.byref(o)) == -1


def test_banded_validation(lib):
    o = salo.make_options()
    f = salo.load().salo_align_batch_banded
    assert f(None, None, None, None, 0, SC, 5, None, None, None, NULL, ctypes.byref(o)) == 0
    assert f(ADDR, ADDR, ADDR, ADDR, 5, SC, -1, ADDR, ADDR, ADDR, NULL, ctypes.byref(o)) == -1
    assert "band" in lib.salo_last_error().decode()
    assert f(ADDR, ADDR, ADDR, ADDR, 5, SC, 65536, ADDR, ADDR, ADDR, NULL,
             ctypes.byref(o)) == -1
    assert f(ADDR, ADDR, ADDR, ADDR, -1, SC, 5, ADDR, ADDR, ADDR, NULL, ctypes.byref(o)) == -1
    assert f(ADDR + 1, ADDR, ADDR, ADDR, 5, SC, 5, ADDR, ADDR, ADDR, NULL,
             ctypes.byref(o)) == -1
    p = salo.make_options(mode="plain")
    assert f(ADDR, ADDR, ADDR, ADDR, 5, SC, 5, ADDR, ADDR, ADDR, NULL, ctypes.byref(p)) == -5
    assert "persistent" in lib.salo_last_error().decode()


def test_trace_validation(lib):
    o = salo.make_options()
    f = salo.load().salo_align_trace
    A = ADDR

    wsbuf = ctypes.create_string_buffer(1024)
    WS = (ctypes.addressof(wsbuf) + 255) & ~255

    def call(n=5, ans=A, off=A, cig=A, ws=WS, wsb=1 << 20, opts=o):
        return f(A, A, A, A, n, SC, ans, ans, ans, ans, ans, off, cig, A, ws, wsb, NULL,
                 ctypes.byref(opts))
    assert f(None, None, None, None, 0, SC, None, None, None, None, None, None, None, None,
             None, 0, NULL, ctypes.byref(o)) == 0
    assert call(ans=None) == -1
    assert call(ans=A + 2) == -1
    assert call(off=A + 4) == -1
    assert call(cig=A + 2) == -1
    assert call(ws=None) == -1
    assert call(ws=WS + 16) == -1
    assert "256-byte" in lib.salo_last_error().decode()
    assert call(wsb=0) == -1
    assert call(opts=salo.make_options(mode="plain")) == -5
    assert call(opts=salo.make_options(cols=32)) == -5
    assert call(n=-1) == -1
