"""Host packer of the library (schedule.cpp), checked on the CPU.

The packer decides, for every chunk of monomials, where each term is staged
in LDS and how the summation is split into pieces.  These tests rebuild the
meaning of the tables independently and check that:
  - every term of a chunk has its own staging slot i*NP + l, where l is a
    piece (0 <= l < NP) and i < the piece's length, and the piece lengths
    add up to the number of terms (so the slots are a bijection onto the
    cells of the pieces),
  - read in piece order, then term order, the slots give the terms ordered
    by output, then by monomial (monomial-order sums),
  - every piece holds one output, pieces tile every output's run, only the
    last piece of a run is short, and first-piece flags sit on output
    boundaries,
  - every group of VG consecutive monomials (VG a power of two) has one
    value term, summed with the value output,
  - padding entries name the dummy variable and the discard slot,
  - the workgroup split covers every chunk exactly once,
for random systems (including empty polynomials and constant monomials)
and several schedules, including chunks that touch more outputs than there
are lanes (then lanes take several pieces).
"""
import ctypes as C
import os
import subprocess
import tempfile

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1201_0499_amd", "csrc")


@pytest.fixture(scope="module")
def probe():
    d = tempfile.mkdtemp(prefix="pe_probe_")
    so = os.path.join(d, "libprobe.so")
    subprocess.run(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", f"-I{CSRC}",
                    os.path.join(ROOT, "tests", "cpp", "schedule_probe.cpp"),
                    os.path.join(CSRC, "schedule.cpp"), "-o", so], check=True)
    L = C.CDLL(so)
    L.probe_build.restype = C.c_void_p
    L.probe_build.argtypes = [C.c_int32, C.c_int32, C.c_int64] + [C.c_void_p] * 4 + \
        [C.c_int] * 4 + [C.c_char_p, C.c_int]
    L.probe_count.restype = C.c_int64
    L.probe_count.argtypes = [C.c_void_p, C.c_int]
    L.probe_copy.argtypes = [C.c_void_p, C.c_int, C.c_void_p]
    L.probe_free.argtypes = [C.c_void_p]
    L.probe_max_stage.argtypes = [C.c_int]
    return L


DT = {0: np.uint32, 1: np.uint16, 3: np.int32, 6: np.uint16, 7: np.uint32,
      8: np.int32, 12: np.int32, 13: np.uint16}
OUT_MASK = (1 << 21) - 1
RUN_SHIFT = 21


def _tables(L, s, lanes, cc, nt, G):
    arrs = [np.ascontiguousarray(s.poly_start, np.int64), np.ascontiguousarray(s.mono_start, np.int64),
            np.ascontiguousarray(s.pos, np.int32), np.ascontiguousarray(s.exp, np.int32)]
    err = C.create_string_buffer(256)
    h = L.probe_build(s.n_vars, s.n_polys, s.n_monos, *[a.ctypes.data for a in arrs],
                      lanes, cc, nt, G, err, 256)
    assert h, err.value
    out = {}
    for w, dt in DT.items():
        n = L.probe_count(h, w)
        a = np.empty(n, dtype=dt)
        if n:
            L.probe_copy(h, w, a.ctypes.data)
        out[w] = a
    out["stage_slots"] = L.probe_count(h, 9)
    out["KP"] = L.probe_count(h, 10)
    out["MC"] = L.probe_count(h, 11)
    out["VG"] = L.probe_count(h, 14)
    L.probe_free(h)
    return out


def _check(s, t, nt, G):
    n = s.n_vars
    KP, MC = t["KP"], t["MC"]
    word, dest = t[0].reshape(-1, KP), t[1].reshape(-1, KP)
    vdest, VG = t[13], t["VG"]
    assert vdest.size == s.n_monos
    assert VG >= 1 and VG & (VG - 1) == 0
    info, plen, pout, g0 = t[3].reshape(-1, 4), t[6], t[7], t[8]
    trash = t["stage_slots"] - 1
    nch = info.shape[0]
    # workgroup split: n_polys*G groups covering all chunks in order
    assert g0.size == s.n_polys * G + 1 and g0[0] == 0 and g0[-1] == nch
    assert np.all(np.diff(g0) >= 0)
    ginfo = t[12].reshape(-1, 8)
    assert ginfo.shape[0] == s.n_polys * G
    for g in range(ginfo.shape[0]):
        assert ginfo[g, 0] == g0[g] and ginfo[g, 1] == g0[g + 1]
        if g0[g] < g0[g + 1]:
            assert np.array_equal(ginfo[g, 2:6], info[g0[g]])
    assert plen.size == pout.size
    covered = []
    piece_base = 0
    for c in range(nch):
        a, nm, p0 = int(info[c, 0]), int(info[c, 1]), int(info[c, 2])
        npc, PL = int(info[c, 3]) & 0xFFFF, (int(info[c, 3]) & 0xFFFFFFFF) >> 16
        assert p0 == piece_base
        piece_base += npc
        assert 1 <= nm <= MC and PL >= 1 and npc >= 1
        assert PL * npc <= trash
        covered.extend(range(a, a + nm))
        # all monomials of a chunk belong to one polynomial
        p = int(np.searchsorted(s.poly_start, a, side="right") - 1)
        assert a + nm <= s.poly_start[p + 1]
        # expected terms: (output, order key, slot)
        expected = []
        for sl in range(nm):
            sidx = a + sl
            b, e = int(s.mono_start[sidx]), int(s.mono_start[sidx + 1])
            for j in range(e - b):
                w = int(word[sidx, j])
                assert w & 0xFFFFFF == s.pos[b + j] and (w >> 24) == s.exp[b + j] - 1
                expected.append((int(s.pos[b + j]), sl * KP + j, int(dest[sidx, j])))
            for j in range(e - b, KP):
                assert int(word[sidx, j]) == n and int(dest[sidx, j]) == trash
            if sl % VG == 0:
                expected.append((n, sl * KP, int(vdest[sidx])))
        T = len(expected)
        lens = plen[p0:p0 + npc].astype(int)
        outs = pout[p0:p0 + npc].astype(np.int64)
        assert np.all(lens >= 1) and np.all(lens <= PL) and int(lens.sum()) == T
        slots = [x[2] for x in expected]
        assert len(set(slots)) == T, "two terms share a slot"
        piece_of = {}
        for o, _, slot in expected:
            i, l = slot // npc, slot % npc
            assert i < lens[l], "slot outside its piece"
            assert piece_of.setdefault(l, o) == o, "a piece mixes outputs"
        order = sorted(expected, key=lambda x: (x[2] % npc, x[2] // npc))
        assert [(o, k) for o, k, _ in order] == sorted((o, k) for o, k, _ in expected)
        l = 0
        while l < npc:
            o = int(outs[l]) & OUT_MASK
            nrun = int(outs[l]) >> RUN_SHIFT
            assert nrun >= 1 and (l == 0 or piece_of[l - 1] != o)
            for j in range(nrun):
                assert int(outs[l + j]) & OUT_MASK == o and piece_of[l + j] == o
                assert j == 0 or int(outs[l + j]) >> RUN_SHIFT == 0
                assert j == nrun - 1 or lens[l + j] == PL
            assert int(lens[l:l + nrun].sum()) == sum(1 for x in expected if x[0] == o)
            l += nrun
    assert covered == list(range(s.n_monos))


CASES = [
    ("tiny", lambda: synth.tiny_workload()[0], [(1, 4, 64, 1), (2, 2, 64, 2), (4, 2, 256, 1)]),
    ("ragged", lambda: synth.regular_system(20, 37, 4, (1, 3), seed=7, n_polys=11),
     [(1, 4, 64, 1), (2, 4, 64, 3), (1, 8, 64, 2)]),
    ("known_root", lambda: synth.known_root_system(10, 13, 5, (1, 3), seed=3)[0],
     [(2, 4, 128, 1), (8, 2, 256, 2)]),
    ("wide", lambda: synth.regular_system(300, 70, 16, (1, 4), seed=9, n_polys=5),
     [(4, 4, 256, 1), (2, 8, 128, 2)]),
]


@pytest.mark.parametrize("name,make,scheds", CASES, ids=[c[0] for c in CASES])
def test_schedule_tables_are_consistent(probe, name, make, scheds):
    s = make()
    for (lanes, cc, nt, G) in scheds:
        t = _tables(probe, s, lanes, cc, nt, G)
        _check(s, t, nt, G)


def test_empty_polynomials_and_too_small_schedule(probe):
    polys = [[], [[(0, 1), (2, 2)], []], []]
    s = synth.system_from_lists(3, polys, [[], [1.0, 2.0], []])
    t = _tables(probe, s, 1, 2, 64, 2)
    _check(s, t, 64, 2)
    arrs = [np.ascontiguousarray(a) for a in (s.poly_start, s.mono_start, s.pos, s.exp)]
    err = C.create_string_buffer(256)
    # a monomial with 2 variables cannot fit 1 lane x 1 variable
    h = probe.probe_build(3, 3, s.n_monos, *[a.ctypes.data for a in arrs], 1, 1, 64, 1, err, 256)
    assert not h and b"more variables" in err.value


def test_staging_capacity_limits_piece_length(probe):
    """With a staging capacity, the packer picks a piece length whose table
    (PL * NP slots + the discard slot) fits, and refuses when none does."""
    s = synth.regular_system(300, 70, 16, (1, 4), seed=9, n_polys=5)
    try:
        free = _tables(probe, s, 4, 4, 256, 1)
        terms_max = 64 * 16 + 64 // free["VG"]  # derivative terms + value terms
        probe.probe_max_stage(terms_max + 1)
        t = _tables(probe, s, 4, 4, 256, 1)
        _check(s, t, 256, 1)
        assert t["stage_slots"] <= terms_max + 1 <= free["stage_slots"] or \
            free["stage_slots"] <= terms_max + 1
        info = t[3].reshape(-1, 4)
        for c in range(info.shape[0]):
            npc, PL = int(info[c, 3]) & 0xFFFF, int(info[c, 3]) >> 16
            assert PL * npc + 1 <= terms_max + 1
        probe.probe_max_stage(100)
        arrs = [np.ascontiguousarray(a) for a in (s.poly_start, s.mono_start, s.pos, s.exp)]
        err = C.create_string_buffer(256)
        h = probe.probe_build(s.n_vars, s.n_polys, s.n_monos, *[a.ctypes.data for a in arrs],
                              4, 4, 256, 1, err, 256)
        assert not h and b"does not fit" in err.value
    finally:
        probe.probe_max_stage(0)
