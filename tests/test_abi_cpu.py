"""Host-side checks of the C-ABI library that need no GPU: it loads, it
exports every function the header declares, and argument validation that
happens before any device work returns the documented codes."""
import ctypes

import numpy as np
import pytest

from paper_2205_07610_amd import binding

AS_ERR_NULL, AS_ERR_SCORING, AS_ERR_ARG = -1, -4, -7


@pytest.fixture(scope="module")
def L():
    return binding.lib()


def test_exports_every_declared_symbol(L):
    names = binding.declared_functions()
    assert "as_align_batch" in names and len(names) >= 4
    for name in names:
        assert hasattr(L, name), name


def test_strerror_and_build_info(L):
    for code in range(0, -8, -1):
        assert binding.strerror(code)
    assert binding.strerror(-99) == "unknown error"
    assert b"gfx950" in L.as_build_info()


def _call(L, *, n_pairs=1, asz=4, alpha=5, beta=2, mode=0, null=None, subst=None):
    sub = np.full((asz, asz), -3, np.int8) if subst is None else subst
    sc = binding.Scoring(asz, sub.ctypes.data_as(ctypes.c_void_p), alpha, beta)
    dummy = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    ptrs = [dummy] * 5
    if null is not None:
        ptrs[null] = ctypes.c_void_p(0)
    return L.as_align_batch(ptrs[0], ptrs[1], ptrs[2], ptrs[3], n_pairs, ctypes.byref(sc), mode,
                            ptrs[4], None)


@pytest.mark.parametrize("which", range(5))
def test_null_pointers(L, which):
    assert _call(L, null=which) == AS_ERR_NULL


def test_null_scoring(L):
    d = ctypes.c_void_p(0x1000)
    assert L.as_align_batch(d, d, d, d, 1, None, 0, d, None) == AS_ERR_NULL


@pytest.mark.parametrize("kw", [dict(asz=1), dict(asz=33), dict(alpha=2, beta=3), dict(beta=-1),
                                dict(mode=3), dict(mode=-1), dict(alpha=20000, beta=0)])
def test_bad_scoring(L, kw):
    assert _call(L, **kw) == AS_ERR_SCORING


def test_bad_n_pairs(L):
    assert _call(L, n_pairs=-1) == AS_ERR_ARG


def test_zero_pairs_is_ok_without_device(L):
    assert _call(L, n_pairs=0) == 0


def test_python_binding_rejects_host_tensors():
    torch = pytest.importorskip("torch")
    t = torch.zeros(4, dtype=torch.uint8)
    o = torch.zeros(2, dtype=torch.int64)
    with pytest.raises(TypeError):
        binding.align_batch(t, o, t, o, np.eye(4, dtype=np.int8), 5, 2, 0,
                            scores_out=torch.zeros(1, dtype=torch.int32), stream=0)


def test_struct_layouts_match_header(tmp_path):
    """The binding's ctypes structs have the C header's field offsets and
    sizes (a host C program built with gcc against include/anyseq_mi.h)."""
    import os
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    structs = {"as_scoring": binding.Scoring, "as_timing": binding.Timing,
               "as_band_stats": binding.BandStats}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "anyseq_mi.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(root, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for field, _ in py._fields_:
            assert got[(cname, field)] == getattr(py, field).offset, (cname, field)


def _fnv_fix(blob, sum_off):
    b = bytearray(blob)
    b[sum_off:sum_off + 4] = b"\0\0\0\0"
    h = 2166136261
    for x in bytes(b):
        h = ((h ^ x) * 16777619) & 0xFFFFFFFF
    b[sum_off:sum_off + 4] = h.to_bytes(4, "little")
    return bytes(b)


def test_variant_tables_blob_round_trip(L):
    """The persisted variant tables: a saved blob restores all three modes'
    tables and measured cell types; a version-1 blob (tables only) still
    loads and clears the cell types; a damaged, truncated or out-of-range
    blob is refused and leaves everything as it was.  Host-only (no device
    work)."""
    prev = [binding.get_variants(m) for m in range(3)]
    prev_h = [binding.half_cells_preference(m) for m in range(3)]
    try:
        tabs = [np.array([0, 1, 2, 3, 4, 5, -1, -1, 2, 2, 4, 4], np.int8),
                np.array([-1] * 12, np.int8),
                np.array([5, 5, 3, 3, 2, 2, 1, 1, 0, 4, 4, -1], np.int8)]
        prefs = [1, -1, 0]
        for m, t in enumerate(tabs):
            binding.set_variants(m, t)
            binding.half_cells_preference(m, prefs[m])
        blob = binding.variant_tables_save()
        assert len(blob) == 68 and blob[:8] == b"ASVARTAB" and blob[8] == 2
        assert list(np.frombuffer(blob[60:63], np.int8)) == prefs and blob[63] == 0

        def clear():
            for m in range(3):
                binding.set_variants(m, None)
                binding.half_cells_preference(m, -1)

        clear()
        binding.variant_tables_load(blob)
        for m, t in enumerate(tabs):
            assert np.array_equal(binding.get_variants(m), t)
            assert binding.half_cells_preference(m) == prefs[m]
        # version 1: the same tables, no cell types, checksum at byte 60
        v1 = bytearray(blob[:64])
        v1[8] = 1
        v1 = _fnv_fix(v1, 60)
        binding.variant_tables_load(v1)
        for m, t in enumerate(tabs):
            assert np.array_equal(binding.get_variants(m), t)
            assert binding.half_cells_preference(m) == -1
        clear()
        bad_sum = bytearray(blob)
        bad_sum[30] ^= 1
        bad_entry = bytearray(blob)
        bad_entry[24] = 9                      # variant 9 does not exist
        bad_pref = bytearray(blob)
        bad_pref[61] = 2                       # cell type 2 does not exist
        bad_pad = bytearray(blob)
        bad_pad[63] = 1
        bad_version = bytearray(blob)
        bad_version[8] = 3
        bads = [bytes(bad_sum), _fnv_fix(bad_entry, 64), _fnv_fix(bad_pref, 64), _fnv_fix(bad_pad, 64),
                _fnv_fix(bad_version, 64), blob[:-1], _fnv_fix(bytearray(blob[:64]), 60)]
        for bad in bads:
            with pytest.raises(binding.AlignError) as e:
                binding.variant_tables_load(bad)
            assert e.value.code == AS_ERR_ARG
            for m in range(3):
                assert np.all(binding.get_variants(m) == -1)
                assert binding.half_cells_preference(m) == -1
        for args in ((3, 0), (-1, 0), (0, 2), (0, -2)):
            with pytest.raises(binding.AlignError):
                binding.half_cells_preference(*args)
    finally:
        for m in range(3):
            binding.set_variants(m, prev[m])
            binding.half_cells_preference(m, prev_h[m])
