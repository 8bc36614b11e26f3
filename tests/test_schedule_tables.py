"""Host packer of the library (schedule.cpp), checked on the CPU.

The packer decides, for every chunk of monomials, where each term is staged
in LDS and how outputs are ranked for the summation.  These tests rebuild
the meaning of the tables independently and check that:
  - every term of a chunk (k derivative terms per monomial, one value term
    per group of VG consecutive monomials, VG a power of two) has its own
    staging slot, and the slots are exactly 0 .. T-1,
  - run_info ranks every output once, by run length, longest first (ties
    by output index), with the right run lengths,
  - the i-th term (in monomial order) of the output of rank j sits at slot
    row_start[i] + j, and row i has exactly as many slots as outputs with
    more than i terms,
  - padding entries name the dummy variable and the discard slot,
  - the workgroup split covers every chunk exactly once,
  - a constant monomial that comes last in its polynomial is in no chunk
    and is named by the polynomial's first group instead,
for random systems (including empty polynomials and constant monomials)
and several schedules.
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


DT = {0: np.uint32, 1: np.uint16, 3: np.int32, 6: np.uint32, 7: np.uint16, 8: np.int32,
      12: np.int32, 13: np.uint16}


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
    out["max_rows"] = L.probe_count(h, 15)
    L.probe_free(h)
    return out


def _check(s, t, nt, G):
    n = s.n_vars
    KP, MC = t["KP"], t["MC"]
    word, dest = t[0].reshape(-1, KP), t[1].reshape(-1, KP)
    vdest, VG = t[13], t["VG"]
    assert vdest.size == s.n_monos
    assert VG >= 1 and VG & (VG - 1) == 0
    info, g0 = t[3].reshape(-1, 4), t[8]
    trash = t["stage_slots"] - 1
    nch = info.shape[0]
    rinfo = t[6].reshape(nch, n + 1) if nch else t[6]
    rstart = t[7].astype(int)
    # workgroup split: n_polys*G groups covering all chunks in order
    assert g0.size == s.n_polys * G + 1 and g0[0] == 0 and g0[-1] == nch
    assert np.all(np.diff(g0) >= 0)
    ginfo = t[12].reshape(-1, 8)
    assert ginfo.shape[0] == s.n_polys * G
    # a constant last monomial of a polynomial is folded: named (index + 1)
    # by the polynomial's first group, in no chunk
    kk = np.diff(s.mono_start)
    folded = []
    for p in range(s.n_polys):
        s0, s1 = int(s.poly_start[p]), int(s.poly_start[p + 1])
        want = s1 if s1 > s0 and kk[s1 - 1] == 0 else 0
        assert ginfo[p * G, 6] == want
        assert np.all(ginfo[p * G + 1:(p + 1) * G, 6] == 0)
        if want:
            folded.append(want - 1)
    assert np.all(ginfo[:, 7] == 0)
    for g in range(ginfo.shape[0]):
        assert ginfo[g, 0] == g0[g] and ginfo[g, 1] == g0[g + 1]
        if g0[g] < g0[g + 1]:
            assert np.array_equal(ginfo[g, 2:6], info[g0[g]])
    covered = []
    for c in range(nch):
        a, y, r0, idx = (int(v) for v in info[c])
        nm, rows = y & 0xFFFF, y >> 16
        assert idx == c and 1 <= nm <= MC and rows <= t["max_rows"]
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
        assert T <= trash
        assert sorted(x[2] for x in expected) == list(range(T)), "slots must be 0 .. T-1"
        # ranking: every output once, by run length (longest first, ties by index)
        lens = np.zeros(n + 1, int)
        for o, _, _ in expected:
            lens[o] += 1
        outs = [int(v) & 0xFFFF for v in rinfo[c]]
        rl = [int(v) >> 16 for v in rinfo[c]]
        assert sorted(outs) == list(range(n + 1))
        assert outs == sorted(range(n + 1), key=lambda o: (-lens[o], o))
        assert rl == [int(lens[o]) for o in outs]
        assert rows == max(rl)
        row = rstart[r0:r0 + rows + 1]
        assert row[0] == 0 and row[-1] == T
        for i in range(rows):
            assert row[i + 1] - row[i] == sum(1 for v in rl if v > i)
        rank = {o: jj for jj, o in enumerate(outs)}
        for o in range(n + 1):
            mine = sorted((k, slot) for oo, k, slot in expected if oo == o)
            for i, (_, slot) in enumerate(mine):
                assert slot == row[i] + rank[o], f"term {i} of output {o}"
    assert sorted(covered + folded) == list(range(s.n_monos))
    assert not set(covered) & set(folded)


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


def test_constant_monomials(probe):
    """Only a constant that comes last in its polynomial is folded: a
    polynomial that is only a constant has no chunk, two trailing constants
    fold the last one, a leading constant stays in its chunk."""
    polys = [[[]], [[(0, 1)], [], []], [[], [(1, 2), (2, 1)]], [[(0, 1), (2, 3)], []]]
    coefs = [[1.0], [1.0, 2.0, 3.0], [4.0, 5.0], [6.0, 7.0]]
    s = synth.system_from_lists(3, polys, coefs)
    for sched in [(1, 2, 64, 1), (2, 2, 64, 2), (1, 4, 64, 3)]:
        t = _tables(probe, s, *sched)
        _check(s, t, sched[2], sched[3])
        ginfo = t[12].reshape(-1, 8)
        G = sched[3]
        assert [int(ginfo[p * G, 6]) for p in range(4)] == [1, 4, 0, 8]
        # the constant-only polynomial has no chunk in any of its groups
        assert np.all(ginfo[0:G, 0] == ginfo[0:G, 1])


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


def test_staging_capacity_is_enforced(probe):
    """With a staging capacity below a chunk's terms + 1, the packer refuses
    the schedule; at exactly that capacity it accepts it."""
    s = synth.regular_system(300, 70, 16, (1, 4), seed=9, n_polys=5)
    try:
        free = _tables(probe, s, 4, 4, 256, 1)
        need = free["stage_slots"]
        probe.probe_max_stage(need)
        t = _tables(probe, s, 4, 4, 256, 1)
        _check(s, t, 256, 1)
        probe.probe_max_stage(need - 1)
        arrs = [np.ascontiguousarray(a) for a in (s.poly_start, s.mono_start, s.pos, s.exp)]
        err = C.create_string_buffer(256)
        h = probe.probe_build(s.n_vars, s.n_polys, s.n_monos, *[a.ctypes.data for a in arrs],
                              4, 4, 256, 1, err, 256)
        assert not h and b"does not fit" in err.value
    finally:
        probe.probe_max_stage(0)


@pytest.mark.parametrize("elem,widest,n,want", [
    (16, 16, 512, 16),    # FP64, n = 512: 128 KiB panel
    (16, 16, 640, 8),     # 16 x 640 x 16 B is exactly 160 KiB: no room for the static arrays
    (32, 8, 640, 4),      # double-double, n = 640
    (16, 16, 1280, 4),
    (32, 8, 2560, 0),     # 2 x 2560 x 32 B = 160 KiB: nothing fits
    (32, 8, 2480, 2),     # 155 KiB + 5 KiB
    (32, 8, 2481, 0),
])
def test_elimination_panel_leaves_room_for_static_lds(probe, elem, widest, n, want):
    """The elimination's panel plus its static arrays (reserved 5 KiB) fit
    in 160 KiB; the width halves until they do, and 0 means unsupported."""
    probe.probe_lu_panel.restype = C.c_int
    probe.probe_lu_panel.argtypes = [C.c_int, C.c_long, C.c_int]
    nb = probe.probe_lu_panel(elem, n, widest)
    assert nb == want
    if nb:
        assert nb * n * elem + 5 * 1024 <= 160 * 1024
