"""The C-ABI library loads and exports every function include/ompd.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

import paper_2406_13881_amd as ompd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "ompd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b(ompd_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("ompd_analyze_cfg", "ompd_analyze_batch", "ompd_submit", "ompd_poll", "ompd_plan_run"):
        assert must in names


@pytest.mark.parametrize("name", declared_functions())
def test_library_exports(name):
    lib = ompd.lib()
    assert hasattr(lib, name), name
    assert ctypes.cast(getattr(lib, name), ctypes.c_void_p).value


def test_no_silent_fallback(monkeypatch, tmp_path):
    """Without the built library the binding raises instead of computing."""
    monkeypatch.setattr(ompd, "_SO", str(tmp_path / "missing.so"))
    monkeypatch.setattr(ompd, "_handle", None)
    with pytest.raises(ompd.OmpdNotBuilt):
        ompd.lib()


def test_ring_slots_flag_matches_header(tmp_path):
    """The binding's F_RING_SLOTS encodes ring sizes exactly as the header's
    OMPD_F_RING_SLOTS macro (compiled with the host C compiler)."""
    import subprocess
    ns = [0, 1, 7, 8, 9, 15, 16, 31, 32, 63, 64, 65, 1000]
    src = tmp_path / "rs.c"
    src.write_text('#include <stdio.h>\n#include "ompd.h"\nint main(void) {\n' +
                   "".join('printf("%%u\\n", (unsigned)OMPD_F_RING_SLOTS(%d));\n' % n for n in ns) +
                   "return 0;\n}\n")
    exe = tmp_path / "rs"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert got == [ompd.F_RING_SLOTS(n) for n in ns]
    assert [ompd.F_RING_SLOTS(n) >> 8 for n in (8, 16, 32, 64)] == [1, 2, 3, 4]


def test_bulk_output_views_match_per_cfg_outputs():
    """The binding's one-buffer-per-output allocation gives every CFG the same zeroed,
    contiguous arrays as allocating them one by one, at the addresses written into the
    result structs, without overlaps."""
    import synth
    cfgs = [synth.c1(i) for i in range(4)] + [synth.random_dag(5, 20, 70, p_loop_entry=0.3)]
    cfgs.append(synth.from_edges([(0, [], []), (0, [], [])], [(0, 1, 0)], 0)[0])   # no variables
    R = (ompd._Res * len(cfgs))()
    outs = ompd._alloc_outputs_many(cfgs, ompd.OUTPUTS, R)
    spans = []
    for i, c in enumerate(cfgs):
        ref = ompd._alloc_outputs(c, ompd.OUTPUTS)
        for k in ompd.OUTPUTS:
            a = outs[i][k]
            assert a.shape == ref[k].shape and a.dtype == ref[k].dtype
            assert a.flags["C_CONTIGUOUS"] and not a.any()
            if a.nbytes:   # (an empty array's address is never written through)
                assert getattr(R[i], ompd._RES_FIELD[k]) == a.ctypes.data
                spans.append((a.ctypes.data, a.ctypes.data + a.nbytes))
    spans.sort()
    assert all(e <= s for (_, e), (s, _) in zip(spans, spans[1:]))
