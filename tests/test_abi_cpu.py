"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
function declared in include/radiate.h, and its host-only planning entry point
validates arguments.  Also checks that the product package never reaches the oracle."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "radiate.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(?:int|void|size_t|const char\*)\s+\**\s*(\w+)\s*\(",
                                 text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2604_09643_amd import _lib, build
    if build.is_stale():
        build.build(verbose=False)
    return _lib.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("radiate_forward", "radiate_adjoint", "loss_and_grad", "ra_create", "ra_destroy",
                 "ra_status", "ra_count_updates"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2604_09643_amd import _lib
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.lib_path()], capture_output=True, text=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if " T " in l)
    assert set(declared_functions()) <= exported
    assert set(_lib.EXPORTS) == set(declared_functions())


def test_library_is_gfx950(lib):
    from paper_2604_09643_amd import _lib
    data = open(_lib.lib_path(), "rb").read()
    assert b"gfx950" in data


def test_scratch_planning_validates(lib):
    from paper_2604_09643_amd import _lib as L
    g = L.Grid(128, 128, 64, (-6.35e-3, -6.35e-3, 6.85e-3), 1e-4)
    s = L.Sampling(1540.0, 40e6, 1024, 0.08e-3)
    n = lib.ra_scratch_bytes(ctypes.byref(g.c()), 128, 64, ctypes.byref(s.cs()))
    assert n >= 64 * 128 * 1024 * 4       # holds at least one signal buffer
    bad = [L.Grid(0, 1, 1, (0, 0, 0), 1e-4), L.Grid(4, 4, 4, (0, 0, 0), -1.0)]
    for b in bad:
        assert lib.ra_scratch_bytes(ctypes.byref(b.c()), 128, 64, ctypes.byref(s.cs())) == 0
    for sb in (L.Sampling(1540.0, 40e6, 0, 1e-4), L.Sampling(1540.0, 40e6, 100, 0.0),
               L.Sampling(1540.0, 40e6, 100, 1e-3)):  # K=0, sigma=0, window > 40 samples
        assert lib.ra_scratch_bytes(ctypes.byref(g.c()), 128, 64, ctypes.byref(sb.cs())) == 0
    assert lib.ra_scratch_bytes(ctypes.byref(g.c()), 0, 64, ctypes.byref(s.cs())) == 0
    # source profiles: unknown kernel ids and power-law exponents nu <= 1/2 are refused
    for kernel, nu, ok in ((1, 1.0, True), (2, 0.75, True), (3, 1.0, True), (4, 1.0, False), (-1, 1.0, False),
                           (2, 0.5, False), (2, float("nan"), False)):
        sk = L.Sampling(1540.0, 40e6, 1024, 0.08e-3, 6.0, kernel, nu)
        assert (lib.ra_scratch_bytes(ctypes.byref(g.c()), 128, 64, ctypes.byref(sk.cs())) > 0) == ok, (kernel, nu)


def test_null_context_is_rejected(lib):
    assert lib.ra_status(None, None) == 1
    assert lib.ra_create(None, 0) == 1


def test_product_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_2604_09643_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                for pat in (r"^\s*(from|import)\s+oracle\b", r"\boracle\.\w+\(", r"liboracle", r"radiate_oracle"):
                    assert not re.search(pat, text, flags=re.M), (f, pat)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asking for several ends with a message and a non-zero code."""
    out = subprocess.run(["python", os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                         timeout=120)
    assert out.returncode != 0
    assert "one GPU" in out.stdout + out.stderr


def test_batch_struct_mirrors_match_the_header(tmp_path):
    """The ctypes mirrors of the batched step's structures (serve.py) have the sizes and field
    offsets that a C compiler gives the header's structs."""
    import shutil
    from paper_2604_09643_amd import serve as S
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    mirrors = {"ra_batch_request": S.CBatchRequest, "ra_batch_info": S.CBatchInfo, "ra_batch": S.CBatch}
    lines = ['#include <cstdio>', '#include <cstddef>', '#include "radiate.h"', 'int main() {']
    for cname, py in mirrors.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append("return 0; }")
    src = tmp_path / "off.cpp"
    src.write_text("\n".join(lines))
    exe = tmp_path / "off"
    subprocess.run([cxx, "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line.strip():
            a, b, v = line.split()
            got[(a, b)] = int(v)
    for cname, py in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_flag_constants_match_the_header():
    """Every RA_* flag and enum value the binding uses equals the header's."""
    import re
    from paper_2604_09643_amd import _lib as L
    hdr = open(os.path.join(ROOT, "include", "radiate.h")).read()
    defines = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define (RA_[A-Z_]+) (\d+)u", hdr)}
    enums = {m.group(1): int(m.group(2)) for m in re.finditer(r"(RA_[A-Z_0-9]+) = (\d+)", hdr)}
    assert {"RA_ACCUMULATE", "RA_LOSS_ON_DEVICE", "RA_SIGNALS_GIVEN"} <= set(defines)
    for name, value in list(defines.items()) + list(enums.items()):
        if hasattr(L, name):
            assert getattr(L, name) == value, name
    for name in ("RA_OK", "RA_EINVAL", "RA_ENOMEM", "RA_ACCUMULATE", "RA_LOSS_ON_DEVICE", "RA_SIGNALS_GIVEN"):
        assert hasattr(L, name), name
