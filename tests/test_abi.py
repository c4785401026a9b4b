"""The C ABI without a GPU: the library loads, exports every function that
include/picsar_hip.h declares, the Python binding's structures have the C
layout, and the argument checks that need no device answer as documented."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "picsar_hip.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pic_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_1407_1810_amd.binding import lib
    return lib()


def test_every_declared_function_is_exported(L):
    from paper_1407_1810_amd.binding import EXPORTED
    names = _declared()
    assert len(names) >= 19
    assert sorted(EXPORTED) == names
    for n in names:
        assert getattr(L, n) is not None, n


def test_struct_layout_matches_the_header(tmp_path):
    from paper_1407_1810_amd.binding import GridDesc, PhysDesc
    src = tmp_path / "layout.c"
    lines = ['#include <stddef.h>', '#include <stdio.h>', f'#include "{HEADER}"', "int main(void) {"]
    for cname, cls in (("pic_grid_desc", GridDesc), ("pic_phys_desc", PhysDesc)):
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0; }"]
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-o", str(exe), str(src)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, cls in (("pic_grid_desc", GridDesc), ("pic_phys_desc", PhysDesc)):
        assert got[(cname, "size")] == C.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


def test_null_arguments_are_rejected_without_a_device(L):
    vp = C.c_void_p
    assert L.pic_create(None, 0, None) == -1
    assert L.pic_step(vp(), 1) == -1
    assert L.pic_get_moments(vp(), 0, None, 0) == -1
    assert L.pic_last_error(vp()) == b"null context"
    out = vp()
    assert L.pic_batch_create(None, 1, None, C.byref(out)) == -1
    assert L.pic_batch_create((vp * 1)(), 0, None, C.byref(out)) == -1
    assert L.pic_batch_create((vp * 1)(), 1, None, None) == -1
    assert L.pic_batch_step(vp(), 1) == -1
    assert L.pic_batch_last_error(vp()) == b"null batch"
    L.pic_destroy(vp())
    L.pic_batch_destroy(vp())


def test_no_device_is_reported_as_a_device_error(L):
    from paper_1407_1810_amd.binding import gpu_available
    if gpu_available():
        pytest.skip("a HIP device is present")
    out = C.c_void_p()
    assert L.pic_create(C.byref(out), 0, None) == -6
    assert not out.value


def _enum_values(prefix):
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    return {m.group(1): int(m.group(2)) for m in re.finditer(r"\b(" + prefix + r"\w+)\s*=\s*(-?\d+)", text)}


def test_moment_kinds_and_status_codes_match_the_header():
    """The binding's moment kinds (including the device Gauss-residual
    reduction and the node charge) and status codes are the header's."""
    from paper_1407_1810_amd import binding as B
    kinds = _enum_values("PIC_MOM_")
    assert kinds == {"PIC_MOM_COUNTS": B.MOM_COUNTS, "PIC_MOM_GAUSS": B.MOM_GAUSS, "PIC_MOM_CARRY": B.MOM_CARRY,
                     "PIC_MOM_STAGE_MS": B.MOM_STAGE_MS, "PIC_MOM_POYNTING": B.MOM_POYNTING,
                     "PIC_MOM_GAUSS_RES": B.MOM_GAUSS_RES, "PIC_MOM_RHO_Q": B.MOM_RHO_Q}
    codes = {k: v for k, v in _enum_values("PIC_E").items() if v < 0}  # PIC_ER.. are field components
    codes["PIC_OK"] = 0
    assert {v: k for k, v in codes.items()} == B.STATUS
    assert len(B.GAUSS_RES_KEYS) == 9


def test_init_grid_is_exported_beside_init(L):
    """pic_init_grid (the boundary's name) and pic_init are the same call:
    both reject a null context without a device."""
    vp = C.c_void_p
    assert L.pic_init_grid(vp(), None, None) == -1
    assert L.pic_init(vp(), None, None) == -1
