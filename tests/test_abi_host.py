"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/pic.h declares, and rejects bad configurations
before touching a device."""
import ctypes as C
import os
import re

import pytest

from paper_2204_12837_amd import inputs as I
from paper_2204_12837_amd import pic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(pic_[a-z_0-9]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    L = pic.lib()
    declared = _declared()
    assert declared, "no declarations found"
    assert set(pic.ENTRY_POINTS) <= declared | {"pic_num_patches"}
    for name in sorted(declared):
        assert hasattr(L, name), name


def _cfg(**over):
    wl = I.workload("uniform64")
    c = pic.make_config(wl)
    for k, v in over.items():
        if isinstance(v, tuple):
            arr = getattr(c, k)
            for i, x in enumerate(v):
                arr[i] = x
        else:
            setattr(c, k, v)
    return c


def test_valid_configs_pass():
    for name in ("uniform64", "uniform1024", "imbalanced", "expansion3d", "adjoint256"):
        c = pic.make_config(I.workload(name))
        rc, msg = pic.validate(c)
        assert rc == pic.PIC_OK, (name, msg)
    assert pic.lib().pic_num_patches(C.byref(pic.make_config(I.workload("uniform1024")))) == 4096
    assert pic.lib().pic_num_patches(C.byref(pic.make_config(I.workload("expansion3d")))) == 8192


def test_workgroup_limits():
    """Multiples of 64 up to 1024 threads, in 2D and 3D."""
    for wl in (I.custom(3, (16, 16, 16), (8, 8, 8), ppc=1), I.custom(2, (32, 32), (8, 8), ppc=1)):
        for wg, ok in ((1024, True), (576, True), (64, True), (1088, False), (1000, False),
                       (0, True), (32, False)):
            rc, msg = pic.validate(pic.make_config(wl, wg_size=wg))
            assert (rc == pic.PIC_OK) == ok, (wg, msg)


def test_x_bins_of_large_patches():
    """A patch whose E/B and J tiles exceed the LDS is cut into x-bins: the
    widest divisor of patch[0] whose tiles fit (auto), or bin_x when given;
    bin_x must divide patch[0], and a patch that fits keeps one bin."""
    bw = lambda wl, bx=0: pic.lib().pic_bin_width(C.byref(pic.make_config(wl, bin_x=bx)))
    small = I.workload("uniform1024")
    assert bw(small) == 16 and bw(small, 8) == 8
    big = I.workload("uniform1024", patch=(64, 128, 1))  # tiles of 64 x 128 cells: 0.63 MB
    assert pic.lib().pic_num_patches(C.byref(pic.make_config(big))) == 128
    b = bw(big)
    # 8 cells: (8+3)(128+3) x 6 + (8+5)(128+5) x 3 doubles = 110 KB
    assert b == 8, b
    assert bw(big, 4) == 4
    rc, msg = pic.validate(pic.make_config(big, bin_x=16))  # 186 KB of tiles
    assert rc == pic.PIC_ERR_ARG and "LDS" in msg, msg
    rc, msg = pic.validate(pic.make_config(big, bin_x=6))
    assert rc == pic.PIC_ERR_ARG and "bin_x" in msg, msg
    rc, msg = pic.validate(pic.make_config(small, bin_x=-2))
    assert rc == pic.PIC_ERR_ARG and "bin_x" in msg, msg
    big3 = I.custom(3, (24, 24, 24), (12, 12, 12), ppc=1)
    assert bw(big3) == 4  # 12-, 6-cell bins do not fit; (4+3)(15)(15) x 6 + (9)(17)(17) x 3
    huge3 = I.custom(3, (32, 32, 32), (32, 32, 32), ppc=1)
    rc, msg = pic.validate(pic.make_config(huge3))
    assert rc == pic.PIC_ERR_ARG and "LDS" in msg, msg


@pytest.mark.parametrize("over,frag", [
    (dict(dim=4), "dim"),
    (dict(shape_order=1), "shape_order"),
    (dict(patch=(5, 8, 1)), "below 6"),
    (dict(patch=(12, 8, 1)), "divide"),
    (dict(dt=1.0), "Courant"),
    (dict(dt=-0.01), "Courant"),
    (dict(d=(0.0, 0.1, 0.1)), "positive"),
    (dict(mode=7), "mode"),
    (dict(wg_size=100), "wg_size"),
    (dict(wg_size=1280), "wg_size"),
    (dict(flags=0x80), "flag"),
    (dict(n=(64, 64, 2)), "2D"),
    (dict(chunk=-1), "chunk"),
    (dict(chunk=300), "chunk"),
])
def test_invalid_configs_rejected(over, frag):
    rc, msg = pic.validate(_cfg(**over))
    assert rc == pic.PIC_ERR_ARG
    assert frag in msg


def test_patch_too_large_for_lds():
    """Tiles of one bin spanning the whole patch do not fit: rejected when
    bin_x asks for that, accepted with narrower automatic x-bins."""
    wl = I.custom(2, (128, 128), (64, 64), ppc=1)
    rc, msg = pic.validate(pic.make_config(wl, bin_x=64))
    assert rc == pic.PIC_ERR_ARG and "LDS" in msg
    assert pic.validate(pic.make_config(wl))[0] == pic.PIC_OK
    wl3 = I.custom(3, (32, 32, 32), (16, 16, 16), ppc=1)
    rc, msg = pic.validate(pic.make_config(wl3, bin_x=16))
    assert rc == pic.PIC_ERR_ARG and "LDS" in msg
    assert pic.lib().pic_bin_width(C.byref(pic.make_config(wl3))) == 1


def test_null_arguments():
    L = pic.lib()
    assert L.pic_validate_config(None, None, 0) == pic.PIC_ERR_ARG
    assert L.pic_num_patches(None) == 0
    assert L.pic_init(None, 0, None) == pic.PIC_ERR_ARG
    L.pic_free(None)  # no-op
    assert L.pic_check(None, None) == pic.PIC_ERR_ARG
    assert L.pic_sync(None, None) == pic.PIC_ERR_ARG
    assert L.pic_last_error(None) == b"null context"


def test_binding_struct_layouts_match_the_header(tmp_path):
    """The ctypes structures have the size and field offsets that a C
    compiler gives the header's structs (a mismatch would pass garbage
    through the ABI silently)."""
    import shutil
    import subprocess

    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = {"pic_config": pic.ConfigC, "pic_species": pic.SpeciesC, "pic_fields": pic.FieldsC,
               "pic_cotangent": pic.CotangentC}
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "pic.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run(["gcc", "-std=c11", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            name, field, val = line.split()
            got[(name, field)] = int(val)
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


@pytest.mark.parametrize("bc", [(3, 0, 0), (0, -1, 0)])
def test_invalid_particle_boundaries_rejected(bc):
    import dataclasses

    wl = dataclasses.replace(I.custom(2, (32, 32), (8, 8), ppc=1), particle_bc=bc)
    rc, msg = pic.validate(pic.make_config(wl))
    assert rc == pic.PIC_ERR_ARG and "particle_bc" in msg, msg
    for ok in ((1, 2, 0), (2, 2, 0), (0, 1, 0)):
        wl = dataclasses.replace(wl, particle_bc=ok)
        assert pic.validate(pic.make_config(wl))[0] == pic.PIC_OK


def test_deterministic_flag_refuses_removing_walls():
    """PIC_FLAG_DETERMINISTIC keeps the dense layout, which cannot delete
    particles: a removing wall is refused; reflecting walls are accepted."""
    import dataclasses

    base = I.custom(2, (32, 32), (8, 8), ppc=1)
    rc, msg = pic.validate(pic.make_config(dataclasses.replace(base, particle_bc=(2, 0, 0)),
                                           flags=pic.FLAG_DETERMINISTIC))
    assert rc == pic.PIC_ERR_ARG and "DETERMINISTIC" in msg, msg
    rc, msg = pic.validate(pic.make_config(dataclasses.replace(base, particle_bc=(1, 0, 0)),
                                           flags=pic.FLAG_DETERMINISTIC))
    assert rc == pic.PIC_OK, msg
    rc, msg = pic.validate(pic.make_config(base, flags=32))
    assert rc == pic.PIC_ERR_ARG


def test_resident_flag_refusals():
    """PIC_FLAG_RESIDENT keeps the slab layout between calls: refused with
    PIC_FLAG_DETERMINISTIC (dense layout) and with removing walls (whose
    counts each call reports); accepted with reflecting walls."""
    import dataclasses

    base = I.custom(2, (32, 32), (8, 8), ppc=1)
    assert pic.validate(pic.make_config(base, flags=pic.FLAG_RESIDENT))[0] == pic.PIC_OK
    rc, msg = pic.validate(pic.make_config(base, flags=pic.FLAG_RESIDENT | pic.FLAG_DETERMINISTIC))
    assert rc == pic.PIC_ERR_ARG and "RESIDENT" in msg, msg
    rc, msg = pic.validate(pic.make_config(dataclasses.replace(base, particle_bc=(0, 2, 0)),
                                           flags=pic.FLAG_RESIDENT))
    assert rc == pic.PIC_ERR_ARG and "removing" in msg, msg
    rc, msg = pic.validate(pic.make_config(dataclasses.replace(base, particle_bc=(1, 0, 0)),
                                           flags=pic.FLAG_RESIDENT))
    assert rc == pic.PIC_OK, msg
