"""Host-side checks of the C ABI that need no GPU: the library loads, it
exports every function include/d3.h declares, and argument validation
returns the documented error codes before any device work."""

import ctypes
import os
import re

import numpy as np
import pytest

import synth
from paper_2310_05279_amd import d3

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "d3.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(d3_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_binding_surface():
    assert set(_declared()) == set(d3.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(d3.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def _create(**kw):
    p = d3.make_params(**kw)
    t = d3._Table(synth.make_table())
    out = ctypes.c_void_p()
    rc = d3.lib().d3_create(ctypes.byref(p), ctypes.byref(t.c), ctypes.byref(out))
    return rc, out


@pytest.mark.parametrize("kw", [dict(r_pot=-1.0), dict(r_cn=0.0), dict(skin=-0.1),
                                dict(r_pot=float("nan")), dict(mode=7),
                                dict(a1=float("inf")), dict(damping=2),
                                dict(damping=1, rs6=0.0), dict(damping=1, rs8=-1.0),
                                dict(s9=float("nan")), dict(s9=1.0, r_atm=6.5),
                                dict(s9=1.0, r_atm=0.0)])
def test_create_rejects_bad_params(kw):
    rc, out = _create(**kw)
    assert rc == d3.D3_ERR_INVALID_ARG
    assert out.value is None
    assert d3.lib().d3_last_error()


def test_create_rejects_bad_tables():
    L = d3.lib()
    p = d3.make_params()
    out = ctypes.c_void_p()
    for mutate in ("n_elem", "n_ref", "asym", "nan"):
        tab = synth.make_table()
        if mutate == "n_ref":
            tab["n_ref"] = tab["n_ref"].copy()
            tab["n_ref"][2] = 6
        if mutate == "asym":
            tab["c6_ref"] = tab["c6_ref"].copy()
            tab["c6_ref"][0, 1, 0, 0] += 1.0
        if mutate == "nan":
            tab["rcov"] = tab["rcov"].copy()
            tab["rcov"][1] = np.nan
        t = d3._Table(tab)
        if mutate == "n_elem":
            t.c.n_elem = 17
        assert L.d3_create(ctypes.byref(p), ctypes.byref(t.c), ctypes.byref(out)) == \
            d3.D3_ERR_INVALID_ARG, mutate
    assert L.d3_create(None, None, ctypes.byref(out)) == d3.D3_ERR_INVALID_ARG
    assert L.d3_create(ctypes.byref(p), None, None) == d3.D3_ERR_INVALID_ARG


def test_null_context_is_rejected_everywhere():
    L = d3.lib()
    assert L.d3_build_neighbors(None, 0, None, None, None, None, None) == d3.D3_ERR_INVALID_ARG
    assert L.d3_coordination(None, None, None, None) == d3.D3_ERR_INVALID_ARG
    assert L.d3_energy_forces_virial(None, None, None, None, None, None, 0, None) == \
        d3.D3_ERR_INVALID_ARG
    assert L.d3_status(None) == d3.D3_ERR_INVALID_ARG
    assert L.d3_evaluate(None, None, None, 0, None) == d3.D3_ERR_INVALID_ARG
    out = d3.d3_outputs()
    assert L.d3_evaluate(None, None, ctypes.byref(out), 0, None) == d3.D3_ERR_INVALID_ARG
    assert L.d3_set_mode(None, 0) == d3.D3_ERR_INVALID_ARG
    assert L.d3_list_stats(None, None) == d3.D3_ERR_INVALID_ARG
    L.d3_destroy(None)  # accepted


def test_error_message_is_per_call():
    L = d3.lib()
    L.d3_status(None)
    assert b"NULL" in L.d3_last_error()


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built library every call raises at once: there is no
    fallback path."""
    monkeypatch.setattr(d3, "LIB_PATH", str(tmp_path / "libd3.so"))
    monkeypatch.setattr(d3, "_lib", None)
    with pytest.raises(OSError, match="not built"):
        d3.lib()
    with pytest.raises(OSError, match="not built"):
        d3.D3(synth.make_table())


def test_package_never_reaches_the_oracle():
    """The product package names nothing under oracle/ (the oracle is test
    infrastructure only), and its sources load no other shared library."""
    pkg = os.path.join(ROOT, "paper_2310_05279_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if not f.endswith((".py", ".hip", ".h", ".cpp", ".c")):
                continue
            src = open(os.path.join(dirpath, f)).read()
            assert not re.search(r"\boracle\b|d3ref", src), f
            if f.endswith(".py"):
                assert len(re.findall(r"ctypes\.CDLL\(", src)) <= 1, f


def test_header_is_plain_c_and_links(tmp_path):
    """include/d3.h compiles as strict C99 (no C++ in the boundary), a C
    program that takes the address of every declared entry point links
    against libd3.so, and the calls that need no GPU behave as from Python:
    the host-only bin planner and the argument checks of d3_create."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    names = _declared()
    src = ["#include <stdio.h>", '#include "d3.h"', "typedef void (*fn)(void);",
           "static fn all[] = {" + ", ".join("(fn)%s" % s for s in names) + "};",
           "int main(void) {",
           "    double cell[9] = {20.5, 0, 0, 3.0, 19.0, 0, 1.0, 2.0, 18.0};",
           "    int32_t pbc[3] = {1, 1, 0}, nb[3], reach[3], nrows = -1, ncn = -1;",
           "    d3_ctx *ctx = NULL;",
           "    int r = d3_bin_plan(cell, pbc, 13.0, 7.0, 500, nb, reach, &nrows, &ncn, NULL, 0);",
           "    if (r != D3_OK) return 1;",
           '    printf("%d %d %d %d %d %d %d %d\\n", nb[0], nb[1], nb[2], reach[0], reach[1],',
           "           reach[2], nrows, ncn);",
           "    r = d3_create(NULL, NULL, &ctx);",
           "    if (r != D3_ERR_INVALID_ARG || ctx != NULL) return 2;",
           '    printf("%s\\n", d3_last_error());',
           "    return (int)(sizeof(all) / sizeof(all[0])) == %d ? 0 : 3;" % len(names),
           "}"]
    c = tmp_path / "use_d3.c"
    c.write_text("\n".join(src) + "\n")
    exe = tmp_path / "use_d3"
    libdir = os.path.dirname(d3.LIB_PATH)
    subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror",
                    "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe),
                    "-L" + libdir, "-ld3", "-Wl,-rpath," + libdir], check=True,
                   capture_output=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stderr
    got = [int(v) for v in out.stdout.split("\n")[0].split()]
    want = d3.d3_bin_plan(np.array([[20.5, 0, 0], [3.0, 19.0, 0], [1.0, 2.0, 18.0]]),
                          (1, 1, 0), 13.0, 7.0, 500)
    assert got[:3] == list(want["nb"]) and got[3:6] == list(want["reach"])
    assert got[6] == len(want["rows"]) and got[7] == want["ncnrows"]
    assert out.stdout.split("\n")[1].strip()  # the per-thread error message


def test_readme_c_example_compiles(tmp_path):
    """The C example in README.md compiles against include/d3.h as strict
    C99 (it stays in step with the header)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    text = open(os.path.join(ROOT, "README.md")).read()
    blocks = re.findall(r"```c\n(.*?)```", text, flags=re.S)
    assert blocks, "README.md has no C example"
    c = tmp_path / "readme_example.c"
    c.write_text(blocks[0])
    subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-c",
                    "-I", os.path.join(ROOT, "include"), str(c), "-o", str(tmp_path / "ex.o")],
                   check=True, capture_output=True)
