"""CPU checks of the C ABI: the library loads, exports every function that
include/pic.h declares, and the binding's ctypes structures have the header's
layout (sizes and offsets printed by a C program compiled against pic.h).
No device call is made."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "pic.h")
SO = os.path.join(ROOT, "paper_1801_00972_amd", "libpic.so")


def _declared():
    txt = open(HDR).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(pic_\w+)\s*\(", txt, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(SO):
        from paper_1801_00972_amd import build
        build.build()
    return C.CDLL(SO)


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    from paper_1801_00972_amd import pic
    assert set(pic.SYMBOLS) == set(names)


def test_struct_layout_matches_header(tmp_path):
    from paper_1801_00972_amd import pic
    src = tmp_path / "layout.c"
    structs = {"pic_config": pic.pic_config, "pic_state_view": pic.pic_state_view,
               "pic_counters": pic.pic_counters, "pic_tuning": pic.pic_tuning,
               "pic_fine_grid": pic.pic_fine_grid}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pic.h"', "int main(void){"]
    for sname, cls in structs.items():
        lines.append(f'printf("{sname} size %zu\\n", sizeof({sname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{sname} {fname} %zu\\n", offsetof({sname}, {fname}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    for line in out:
        if not line:
            continue
        sname, field, val = line.split()
        cls = structs[sname]
        if field == "size":
            assert C.sizeof(cls) == int(val), sname
        else:
            assert getattr(cls, field).offset == int(val), f"{sname}.{field}"


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1801_00972_amd import pic
    monkeypatch.setattr(pic, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(pic, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        pic.lib()


def test_workload_configs_are_consistent():
    from paper_1801_00972_amd import workloads as W
    from paper_1801_00972_amd.pic import make_config
    for wl in (W.small_fp64(), W.small_fp32r(), W.full_fp64(), W.full_fp64("fp32r")):
        c, keep = make_config(wl)
        g = keep[0]
        assert c.n_grains == len(g)
        c3 = int(wl["cutoff"])
        for p in g:
            k = int(p[2] // 1)
            assert k - c3 >= 0 and k + c3 + 1 <= wl["nz"]
        if len(g) > 1:
            d = ((g[:, None, :] - g[None, :, :]) ** 2).sum(-1) ** 0.5
            assert d[d > 0].min() >= 200e-6 / wl["dx"] - 1e-9
    assert W.small_fp64()["grain_pos"].tolist() == [[8.0, 8.0, 16.0]]


def test_weight_of_128_or_more_is_rejected(lib):
    """The fixed-point deposit forms Qp * f24 in int64 with f24 < 2^24, so the
    macro charge Qp = w 2^32 must stay below 2^39 (w < 128): the oracle's
    derivation refuses it, and pic_init returns PIC_ECONFIG before any device
    call (so this runs without a GPU)."""
    import oracle
    from paper_1801_00972_amd import pic
    from paper_1801_00972_amd import workloads as W
    wl = W.small_fp64()
    n_at = 128.0 * wl["ppc"] / wl["dx"] ** 3
    L = pic.lib()
    for n0, ok in ((n_at * (1 - 1e-9), True), (n_at, False), (n_at * 1.5, False)):
        o = oracle.Oracle(dict(wl, n0=n0))
        if ok:
            d = o.derived()
            assert d["Qp"] < 2 ** 39 and 2 ** 39 - d["Qp"] < 2 ** 39 * 1e-8
            continue
        with pytest.raises(ValueError):
            o.derived()
        c, keep = pic.make_config(dict(wl, n0=n0))
        out = C.c_void_p()
        rc = L.pic_init(C.byref(c), 1, None, C.byref(out))
        assert rc == pic.PIC_ECONFIG
        assert not out.value
        assert "below 128" in pic.pic_last_error(None)
