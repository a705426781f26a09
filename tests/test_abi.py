"""Host-side checks of the C ABI: the library builds, loads and exports every
symbol include/ibr.h declares; host-only calls behave (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ibr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ibr_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1505_07865_amd import ibr
    if not os.path.exists(ibr.LIB_PATH):
        from paper_1505_07865_amd import build
        build.build()
    return ibr.load()


def test_exports_match_header(lib):
    from paper_1505_07865_amd import ibr
    decl = _declared()
    assert decl, "no declarations parsed"
    for name in decl:
        assert hasattr(lib, name), name
    assert sorted(ibr.EXPORTS) == decl


def test_default_params_and_status(lib):
    from paper_1505_07865_amd import ibr
    p = ibr.Params()
    lib.ibr_default_params(ctypes.byref(p))
    assert p.dim == 3 and p.restart == 100 and p.n_s == 2 and p.rtol == 1e-8 and p.walls == 0 and p.advection == 0
    assert p.mobility == 2          # IBR_MOB_AUTO
    assert lib.ibr_status_string(0) == b"ok"
    assert lib.ibr_status_string(5).startswith(b"mobility")


def test_params_layout_matches_header(tmp_path):
    """The binding's ibr_params / ibr_info mirror the header's structs: size
    and every field offset, as a C compiler lays them out."""
    import shutil
    import subprocess
    from paper_1505_07865_amd import ibr
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ibr.h"', 'int main(void) {']
    for st, cls in (("ibr_params", ibr.Params), ("ibr_info", ibr.Info)):
        lines.append('  printf("%s %%zu\\n", sizeof(%s));' % (st, st))
        for name, _ in cls._fields_:
            lines.append('  printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (st, name, st, name))
    lines.append('  return 0; }')
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(root, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                  text=True).stdout.splitlines())
    for st, cls in (("ibr_params", ibr.Params), ("ibr_info", ibr.Info)):
        assert int(got[st]) == ctypes.sizeof(cls), st
        for name, _ in cls._fields_:
            assert int(got[st + "." + name]) == getattr(cls, name).offset, (st, name)


def test_invalid_params_rejected_before_device_work(lib):
    from paper_1505_07865_amd import ibr
    for bad in (dict(dim=4), dict(n=48), dict(h=0.0), dict(eta=-1.0), dict(rho=1.0, dt=0.0), dict(n_s=0),
                dict(rtol=0.0), dict(precision=7), dict(walls=3), dict(walls=-1), dict(advection=2), dict(advection=-1),
                dict(mobility=3), dict(mobility=-1)):
        p = ibr.default_params(**bad)
        ctx = ctypes.c_void_p()
        assert lib.ibr_create(ctypes.byref(p), ctypes.byref(ctx)) == 1, bad
        assert not ctx.value


def test_footprint_grows_with_grid(lib):
    from paper_1505_07865_amd import ibr
    one = (ctypes.c_int * 1)(200)
    f = [lib.ibr_footprint_bytes(ctypes.byref(ibr.default_params(n=n, h=1.0 / n)), 1, one) for n in (32, 64, 128)]
    assert f[0] < f[1] < f[2]
    fm = lib.ibr_footprint_bytes(ctypes.byref(ibr.default_params(n=128, h=1.0 / 128, precision=1)), 1, one)
    assert fm < f[2]
    # the slit channel keeps every multigrid level down to 4^3 in global memory as well
    fw = lib.ibr_footprint_bytes(ctypes.byref(ibr.default_params(n=128, h=1.0 / 128, walls=1)), 1, one)
    assert fw > f[2]


def test_footprint_counts_each_body_block(lib):
    """The mobility blocks are sized per body: 600 markers as one body hold
    one block of (3 * 600)^2 doubles per buffer (its leading dimension padded
    to a multiple of 16), three bodies of 200 three blocks of (3 * 200)^2;
    invalid counts give 0."""
    from paper_1505_07865_amd import ibr
    p = ibr.default_params(n=64, h=1.0 / 64)
    one = lib.ibr_footprint_bytes(ctypes.byref(p), 1, (ctypes.c_int * 1)(600))
    three = lib.ibr_footprint_bytes(ctypes.byref(p), 3, (ctypes.c_int * 3)(200, 200, 200))
    pad = lambda r: (r + 15) // 16 * 16
    assert one - three == 4 * 8 * (pad(1800) ** 2 - 3 * pad(600) ** 2)
    assert ibr.footprint_bytes([200, 200, 200], n=64, h=1.0 / 64) == three
    assert lib.ibr_footprint_bytes(ctypes.byref(p), 2, None) == 0
    assert lib.ibr_footprint_bytes(ctypes.byref(p), 1, (ctypes.c_int * 1)(-1)) == 0
    assert lib.ibr_footprint_bytes(None, 1, (ctypes.c_int * 1)(10)) == 0


def test_oracle_is_not_imported_by_product():
    pkg = os.path.join(ROOT, "paper_1505_07865_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, fn


def test_timer_classes_known_to_library_and_bench(lib):
    """Every live timer class the binding lists is one the library accepts
    (enable, read back empty, switch off: no launch, so no device work), the
    header documents it, and bench.py has a sampling stride for it; unknown
    classes and negative strides are rejected."""
    import importlib.util
    from paper_1505_07865_amd import ibr
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    header = open(os.path.join(ROOT, "include", "ibr.h")).read()
    for name in ibr.TIMERS:
        ibr.timer_enable(name, 3)
        assert ibr.timer_read(name) == {"ms": 0.0, "launches": 0, "bytes": 0.0}
        ibr.timer_enable(name, 0)
        assert '"%s"' % name in header, name
        assert bench.TIMER_STRIDE.get(name, 0) > 0, name
    assert set(bench.TIMER_STRIDE) == set(ibr.TIMERS)
    with pytest.raises(ibr.IbrError):
        ibr.timer_enable("no_such_kernel", 1)
    with pytest.raises(ibr.IbrError):
        ibr.timer_enable("rb_fine", -1)
