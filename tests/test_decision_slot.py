"""The host side of the C-phase decision hand-off (csrc/decision.h), compiled
with the host compiler and fed whole and torn slots.

The decision kernel writes six 32-bit payload words, each paired with the
call's sequence number in one aligned 8-byte word.  A slot whose words come
partly from an earlier call (a store that has not landed yet), or whose
contents do not fit the chunk that was evaluated, must be refused, so the
host never commits to a date the device did not decide.
"""
import ctypes as C
import math
import os
import struct
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "paper_1304_4334_amd", "csrc")

HARNESS = r"""
#include "decision.h"
extern "C" int parse(const uint32_t *w, uint32_t seq, int64_t t, int64_t t1, int64_t *tc,
                     double *rss, int32_t *ends, int32_t *below, int32_t *flags) {
  smc::DecisionSlot s;
  for (int i = 0; i < 12; ++i) s.w[i] = w[i];
  smc::StopInfo o{};
  if (!smc::read_decision(&s, seq, t, t1, &o, flags)) return 0;
  *tc = o.t_commit; *rss = o.rss; *ends = o.ends; *below = o.below;
  return 1;
}
"""


@pytest.fixture(scope="module")
def parse(tmp_path_factory):
    d = tmp_path_factory.mktemp("slot")
    src, lib = d / "h.cpp", d / "libh.so"
    src.write_text(HARNESS)
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I", HEADER_DIR, str(src),
                    "-o", str(lib)], check=True)
    L = C.CDLL(str(lib))
    L.parse.restype = C.c_int
    L.parse.argtypes = [C.POINTER(C.c_uint32), C.c_uint32, C.c_int64, C.c_int64,
                        C.POINTER(C.c_int64), C.POINTER(C.c_double), C.POINTER(C.c_int32),
                        C.POINTER(C.c_int32), C.POINTER(C.c_int32)]

    def call(words, seq, t, t1):
        arr = (C.c_uint32 * 12)(*words)
        tc, rss = C.c_int64(0), C.c_double(0)
        ends, below, fl = C.c_int32(0), C.c_int32(0), C.c_int32(0)
        ok = L.parse(arr, seq, t, t1, C.byref(tc), C.byref(rss), C.byref(ends), C.byref(below),
                     C.byref(fl))
        return (tc.value, rss.value, ends.value, below.value, fl.value) if ok else None

    return call


def slot_words(seq, t_commit, rss, flags, ends, below, seqs=None):
    rb = struct.unpack("<Q", struct.pack("<d", rss))[0]
    tc = t_commit & (2 ** 64 - 1)
    payload = [tc & 0xFFFFFFFF, tc >> 32, rb & 0xFFFFFFFF, rb >> 32, flags & 0xFFFFFFFF,
               (ends & 1) | ((below & 1) << 1)]
    seqs = seqs or [seq] * 6
    out = []
    for i in range(6):
        out += [seqs[i], payload[i]]
    return out


def test_whole_slot_is_read(parse):
    w = slot_words(7, 1234, 0.4375, 2, 1, 1)
    assert parse(w, 7, 1200, 1300) == (1234, 0.4375, 1, 1, 2)
    # a phase that runs on: no stop in the chunk, committed at its end
    w = slot_words(8, 1300, 0.75, 0, 0, 0)
    assert parse(w, 8, 1200, 1300) == (1300, 0.75, 0, 0, 0)
    # dates beyond 2^32 travel in two words
    big = (1 << 33) + 5
    assert parse(slot_words(9, big, 0.1, 0, 1, 1), 9, big - 10, big)[0] == big


@pytest.mark.parametrize("stale", range(6))
def test_slot_with_a_stale_word_is_refused(parse, stale):
    """One 8-byte word still holds the previous call's contents (its store has
    not landed): the pair's sequence number gives it away."""
    old = slot_words(6, 1100, 0.9, 0, 0, 0)
    new = slot_words(7, 1234, 0.4375, 0, 1, 1)
    torn = list(new)
    torn[2 * stale:2 * stale + 2] = old[2 * stale:2 * stale + 2]
    assert parse(torn, 7, 1200, 1300) is None
    assert parse(new, 7, 1200, 1300) is not None


def test_torn_halves_are_refused(parse):
    """The first 16 bytes from the new call, the rest from the previous one
    (a 16-byte store split in two), and the reverse."""
    old = slot_words(6, 1100, 0.9, 0, 0, 0)
    new = slot_words(7, 1234, 0.4375, 0, 1, 1)
    assert parse(new[:4] + old[4:], 7, 1200, 1300) is None
    assert parse(old[:4] + new[4:], 7, 1200, 1300) is None
    assert parse(new[:8] + old[8:], 7, 1200, 1300) is None


@pytest.mark.parametrize("tc,rss,ends,below", [
    (1200, 0.3, 1, 1),        # not after the chunk's start
    (1301, 0.3, 1, 1),        # beyond the chunk
    (1250, math.nan, 1, 1),   # not a ratio
    (1250, -0.1, 1, 1),
    (1250, 1.5, 0, 0),
    (1250, 0.3, 0, 1),        # below the threshold, but the phase goes on
])
def test_inconsistent_decision_is_refused(parse, tc, rss, ends, below):
    assert parse(slot_words(7, tc, rss, 0, ends, below), 7, 1200, 1300) is None


def test_bad_flag_bits_are_refused(parse):
    w = slot_words(7, 1250, 0.3, 0, 1, 1)
    w[11] = 5
    assert parse(w, 7, 1200, 1300) is None
