"""The C ABI library loads, exports every entry point declared in
include/ddamg.h, and validates arguments before any HIP call (no GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ddamg.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"^\s*typedef[^;]*;", "", src, flags=re.M)  # function-pointer types are not entry points
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def dd():
    import paper_1512_04506_amd as dd
    return dd


def test_header_declares_the_entry_points():
    names = _declared_functions()
    for n in ("mg_setup", "mg_apply", "dirac_apply", "coarse_apply", "solve", "ddamg_create", "ddamg_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol(dd):
    names = _declared_functions()
    out = subprocess.run(["nm", "-D", "--defined-only", dd.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if " T " in line)
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    lib = ctypes.CDLL(dd.LIB_PATH)
    for n in names:
        assert hasattr(lib, n)
    assert set(dd.EXPORTS) == set(names)


def test_default_params(dd):
    p = dd.default_params()
    assert tuple(p.block) == (4, 4, 4, 4)
    assert p.ntv == 24 and p.nu == 3 and p.n_mr == 4 and p.n_setup == 3
    assert p.coarse_tol == 0.05 and p.coarse_restart == 30 and p.coarse_maxit == 300
    assert p.outer_restart == 20 and p.prec == dd.MIXED16 and p.max_rhs == 12
    assert dd.validate_params(p) == (0, "")


@pytest.mark.parametrize("change,needle", [
    (dict(block=(3, 4, 4, 4)), "divide"),
    (dict(L=(12, 8, 8, 8)), "even"),
    (dict(L=(8, 8, 8, 4), block=(4, 4, 4, 4)), "even"),
    (dict(block=(1, 1, 1, 1), L=(8, 8, 8, 8), ntv=8), "aggregates too small"),
    (dict(ntv=0), "ntv"),
    (dict(ntv=33), "ntv"),
    (dict(prec=7), "precision"),
    (dict(max_rhs=0), "max_rhs"),
    (dict(max_rhs=65), "max_rhs"),
    (dict(coarse_restart=0), "restart"),
    (dict(outer_restart=65), "restart"),
    (dict(coarse_tol=0.0), "coarse_tol"),
    (dict(nu=-1), "non-negative"),
    (dict(L=(16, 16, 16, 16), block=(8, 8, 4, 2)), "256"),
    (dict(m0=float("nan")), "finite"),
])
def test_validation_rejects(dd, change, needle):
    p = dd.default_params(**change)
    rc, msg = dd.validate_params(p)
    assert rc == -1
    assert needle in msg


def test_create_rejects_before_any_hip_call(dd):
    """Invalid parameters and NULL pointers come back as codes on a machine
    without a GPU, i.e. before the HIP runtime is touched."""
    lib = dd.lib
    h = ctypes.c_void_p()
    p = dd.default_params(block=(3, 4, 4, 4))
    rc = lib.ddamg_create(ctypes.byref(p), ctypes.c_void_p(16), None, ctypes.byref(h))
    assert rc == -1 and not h.value
    assert b"divide" in lib.ddamg_last_error(None)
    p = dd.default_params()
    rc = lib.ddamg_create(ctypes.byref(p), None, None, ctypes.byref(h))
    assert rc == -1
    assert b"gauge" in lib.ddamg_last_error(None)
    assert lib.ddamg_destroy(None) == -1
    assert lib.mg_setup(None, None) == -1
    assert lib.solve(None, None, None, 1, 1e-10, None) == -1
    assert lib.dirac_apply(None, None, None, 1, 0) == -1
    assert lib.coarse_apply(None, None, None, 1) == -1
    assert lib.mg_apply(None, None, None, 1) == -1
    assert lib.ddamg_volume(None) == -1


def test_set_allocator_arguments(dd):
    """Exactly one of the two hooks NULL is rejected; both NULL restores
    the default (no GPU involved)."""
    a = dd.ALLOC_FN(lambda n, user: None)
    assert dd.lib.ddamg_set_allocator(a, dd.FREE_FN(), None) == -1
    assert b"both" in dd.lib.ddamg_last_error(None)
    assert dd.lib.ddamg_set_allocator(dd.ALLOC_FN(), dd.FREE_FN(), None) == 0
    with pytest.raises(ValueError):
        dd.set_allocator(lambda n: 0, None)
    dd.set_allocator()


def test_import_rejects_null_and_missing_setup(dd):
    assert dd.lib.ddamg_import_tv(None, None) == -1
    assert dd.lib.ddamg_import_coarse(None, None) == -1


def test_switches_reject_null_context(dd):
    """The per-context switches return the argument error for a NULL context
    before touching anything (no GPU needed)."""
    for name in ("ddamg_set_coarse_host_sync", "ddamg_set_graphs", "ddamg_set_coarse_single_kernel",
                 "ddamg_set_kernel_timing"):
        for on in (0, 1):
            assert getattr(dd.lib, name)(None, on) == -1, name


def test_params_struct_matches_the_header(dd, tmp_path):
    """The ctypes mirror of ddamg_params has the C struct's size and field
    offsets (a C program compiled against the header prints them), and the
    binding follows the header's ABI version."""
    import shutil
    if shutil.which("gcc") is None:
        pytest.skip("needs gcc")
    fields = [f for f, _ in dd.Params._fields_]
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "ddamg.h"\nint main(void) {\n'
                   '  printf("%d %zu\\n", DDAMG_ABI_VERSION, sizeof(ddamg_params));\n' +
                   "".join('  printf("%%zu\\n", offsetof(ddamg_params, %s));\n' % f for f in fields) +
                   "  return 0;\n}\n")
    exe = str(tmp_path / "layout")
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", exe], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    assert int(out[0]) == dd.ABI_VERSION
    assert int(out[1]) == ctypes.sizeof(dd.Params)
    for f, off in zip(fields, out[2:]):
        assert getattr(dd.Params, f).offset == int(off), f
    assert fields[-1] == "seed" and dd.default_params().seed == 0


def test_setup_without_start_vectors_needs_only_a_context(dd):
    """mg_setup(ctx, NULL) is the seeded start (Philox4x32-10 on the device
    keyed by params.seed), not an error: with no context it is still
    refused before any HIP call."""
    assert dd.lib.mg_setup(None, None) == -1
    src = open(HEADER).read()
    assert "tv_init == NULL" in src and "Philox4x32-10" in src
