"""CPU checks of the C-ABI library: it loads, exports every function that
include/pibm.h declares, sizes workspaces and rejects bad configurations
without touching a GPU (no compute call is made here)."""
import ctypes as C
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    from paper_1407_6704_amd import pibm
    try:
        pibm.load()
    except RuntimeError:
        from paper_1407_6704_amd import build
        build.build()
    return pibm


def test_exports_every_declared_symbol(P):
    lib = P.load()
    names = P.header_symbols()
    assert len(names) >= 17
    for n in names:
        assert hasattr(lib, n), n
    # nm view as well: the symbols are real exports of the shared object
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", P.LIB_PATH], capture_output=True, text=True).stdout
    for n in names:
        assert f" T {n}" in out, n


def test_workspace_bytes_and_validation(P):
    lib = P.load()
    ok = P.make_config(lattice=9, n=(64, 32, 1), tau=0.8)
    b0 = lib.pibm_workspace_bytes(C.byref(ok), 0)
    b1 = lib.pibm_workspace_bytes(C.byref(ok), 100)
    assert b0 > 9 * 64 * 32 * 4 * 2 and b1 > b0
    fp16 = P.make_config(lattice=19, n=(16, 16, 16), tau=0.8, storage="fp16")
    fp32 = P.make_config(lattice=19, n=(16, 16, 16), tau=0.8)
    assert lib.pibm_workspace_bytes(C.byref(fp16), 0) < lib.pibm_workspace_bytes(C.byref(fp32), 0)
    bad = [
        dict(tau=0.5), dict(tau=0.3), dict(n_sub=0), dict(lattice=27), dict(interp=2), dict(contact="hertz", young=0.0),
        dict(contact="hertz", poisson=0.5), dict(contact=6), dict(contact="hertz_mindlin_microslip", young=0.0),
        dict(contact="hertz_mindlin", friction=-0.1), dict(contact="hertz_mindlin", young=-1.0), dict(n=(8, 8, 2)),
        dict(bin_log2=5), dict(max_candidates=0), dict(restitution=0.0), dict(periodic=(1, 0, 0)),
    ]
    for kw in bad:
        args = dict(lattice=9, n=(8, 8, 1), tau=0.8)
        args.update(kw)
        cfg = P.make_config(**args)
        assert lib.pibm_workspace_bytes(C.byref(cfg), 10) == 0, kw
    # a periodic lattice without particles is allowed (Poiseuille channel)
    per = P.make_config(lattice=9, n=(1, 8, 1), periodic=(1, 0, 0))
    assert lib.pibm_workspace_bytes(C.byref(per), 0) > 0
    # ABI version is checked
    v = P.make_config()
    v.abi_version = 99
    assert lib.pibm_workspace_bytes(C.byref(v), 0) == 0
    # create refuses a too-small workspace and a bad config before any GPU call
    ctx = C.c_void_p()
    assert lib.pibm_create(C.byref(ok), 0, None, 0, None, C.byref(ctx)) == 1
    badc = P.make_config(tau=0.4)
    assert lib.pibm_create(C.byref(badc), 0, None, 0, None, C.byref(ctx)) == 2


def test_config_struct_layout(P, tmp_path):
    """The ctypes mirrors have the C structs' sizes and field offsets, as a C
    compiler lays them out from include/pibm.h."""
    import subprocess

    lines = []
    for cname, py in (("pibm_config", P.Config), ("pibm_diag", P.Diag)):
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "pibm.h"\nint main(void) {\n'
                   + "\n".join(lines) + "\nreturn 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(l.rsplit(" ", 1) for l in subprocess.check_output([str(exe)], text=True).splitlines())
    for cname, py in (("pibm_config", P.Config), ("pibm_diag", P.Diag)):
        assert int(got[f"{cname} size"]) == C.sizeof(py)
        for f in py._fields_:
            assert int(got[f"{cname} {f[0]}"]) == getattr(py, f[0]).offset, (cname, f[0])


def test_single_hip_runtime_in_process(P):
    """Loading the library before torch must still leave exactly one HIP and
    one HSA runtime mapped (the library binds to torch's copy)."""
    import subprocess
    import sys

    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_1407_6704_amd import pibm\n"
        "pibm.load()\n"
        "maps = open('/proc/self/maps').read().splitlines()\n"
        "hip = {l.split()[-1] for l in maps if 'libamdhip64' in l}\n"
        "hsa = {l.split()[-1] for l in maps if 'libhsa-runtime64' in l}\n"
        "print(len(hip), len(hsa))\n" % ROOT
    )
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split() == ["1", "1"], out.stdout
