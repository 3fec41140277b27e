"""The C ABI: exported symbols and struct layouts (CPU only, no compute calls)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2405_04229_amd import cphot

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def declared_functions():
    names = []
    for h in HEADERS:
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?\w[\w\s\*]*?\b(cphot_\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_headers_declare_entry_points():
    names = declared_functions()
    for want in ("cphot_make_atmosphere", "cphot_destroy_atmosphere", "cphot_propagate", "cphot_version"):
        assert want in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(cphot.LIB_PATH):
        pytest.skip("libcphot.so not built")
    out = subprocess.run(["nm", "-D", "--defined-only", cphot.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (cphot_\w+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing


def test_library_loads_without_gpu():
    if not os.path.exists(cphot.LIB_PATH):
        pytest.skip("libcphot.so not built")
    L = cphot.lib()
    assert L.cphot_version() == cphot.ABI_VERSION
    header = open(os.path.join(os.path.dirname(__file__), "..", "include", "cphot.h")).read()
    assert int(re.search(r"#define CPHOT_ABI_VERSION (\d+)", header).group(1)) == cphot.ABI_VERSION
    assert L.cphot_status_string(-1) == b"invalid argument"


STRUCTS = {"cphot_atmosphere_desc": cphot.AtmosphereDesc, "cphot_segments": cphot.Segments,
           "cphot_detector": cphot.Detector, "cphot_bins": cphot.Bins, "cphot_surrogate_desc": cphot.SurrogateDesc,
           "cphot_tuning": cphot.Tuning, "cphot_host_segments": cphot.HostSegments,
           "cphot_table_desc": cphot.TableDesc}


def test_ctypes_layouts_match_header(tmp_path):
    """Offsets and sizes from a C program compiled against the header equal the
    binding's ctypes layouts."""
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADERS[0]}"', "int main(void){"]
    for cname, st in STRUCTS.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in st._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append('printf("cphot_photon_record size %zu\\n", sizeof(cphot_photon_record));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-o", str(exe), str(src)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        s, f, v = line.split()
        got[(s, f)] = int(v)
    for cname, st in STRUCTS.items():
        assert got[(cname, "size")] == ctypes.sizeof(st), cname
        for fname, _ in st._fields_:
            assert got[(cname, fname)] == getattr(st, fname).offset, (cname, fname)
    assert got[("cphot_photon_record", "size")] == cphot.RECORD_BYTES
