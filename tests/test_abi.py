"""The C-ABI library loads and exports every symbol include/lof.h declares, and
argument validation rejects bad parameters before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    with open(os.path.join(ROOT, "include", "lof.h")) as f:
        src = f.read()
    return sorted(set(re.findall(r"^\s*(?:lof_status|const char\*)\s+(lof_\w+)\s*\(", src, re.M)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("lof_create", "lof_flag_blocks", "lof_history_update", "lof_destroy"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_1701_08197_amd import _native as N
    if not N.lib_exists():
        pytest.skip("liblof.so not built")
    L = N.load()
    for s in declared_symbols():
        assert hasattr(L, s), s
    assert set(N.EXPORTED) == set(declared_symbols())


def test_struct_layouts_match_header(tmp_path):
    """ctypes mirrors agree with the C compiler on every field offset and size."""
    import shutil
    import subprocess
    from paper_1701_08197_amd import _native as N
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"lof_params": N.LofParams, "lof_block": N.LofBlock, "lof_block_stats": N.LofBlockStats,
               "lof_tuning": N.LofTuning}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lof.h"', "int main(void){"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = dict(l.split() for l in subprocess.check_output([str(exe)], text=True).splitlines())
    for cname, cls in structs.items():
        assert int(out[cname]) == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert int(out[f"{cname}.{fname}"]) == getattr(cls, fname).offset, (cname, fname)


def test_defaults_and_invalid_params_rejected_without_device():
    from paper_1701_08197_amd import _native as N
    if not N.lib_exists():
        pytest.skip("liblof.so not built")
    L = N.load()
    p = N.LofParams()
    assert L.lof_default_params(ctypes.byref(p)) == N.LOF_OK
    assert (p.start_threshold, p.p, p.sensitivity, p.n_levels) == (6.0, 1.5, 1.0, 7)
    assert (p.sir_eta_num, p.sir_eta_den) == (1, 5)
    h = ctypes.c_void_p()
    for field, val in (("n_levels", 0), ("n_levels", 8), ("sir_eta_num", 6), ("max_channels", 2000),
                       ("history_len", 0), ("max_streams", 0)):
        q = N.LofParams.from_buffer_copy(p)
        setattr(q, field, val)
        assert L.lof_create(ctypes.byref(q), 0, ctypes.byref(h)) == N.LOF_ERR_INVALID
        assert h.value is None
        assert L.lof_last_error(None)
    assert L.lof_flag_blocks(None, None, 0, None, None) == N.LOF_ERR_INVALID
    assert L.lof_history_update(None, None, 0, None) == N.LOF_ERR_INVALID
    assert L.lof_destroy(None) == N.LOF_OK


def test_service_descriptor_view_matches_struct():
    """The streaming service writes descriptor tables through a numpy view."""
    import numpy as np
    from paper_1701_08197_amd import _native as N
    from paper_1701_08197_amd.serve import BLOCK_DTYPE
    names = ["data", "flags", "dstride", "fstride", "C", "T", "dtype", "sid"]
    for (cname, _), nname in zip(N.LofBlock._fields_, names):
        assert BLOCK_DTYPE.fields[nname][1] == getattr(N.LofBlock, cname).offset
    assert BLOCK_DTYPE.itemsize == np.dtype(np.uint8).itemsize * 48
