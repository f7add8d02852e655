"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/btpcg.h, and validates arguments before any HIP call."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2503_15269_amd as bt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "btpcg.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(bt.LIB_PATH):
        pytest.skip("libbtpcg.so not built (run python -m paper_2503_15269_amd.build)")
    return bt.load_library()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(bt_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_binding_symbols():
    assert sorted(bt.exported_symbols()) == declared_functions()


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_strerror_and_defaults(lib):
    assert bt.strerror(bt.OK) == "ok"
    assert "workspace" in bt.strerror(bt.ENOSPACE)
    p = bt._Params()
    lib.bt_default_params(ctypes.byref(p))
    assert (p.a, p.b, p.m, p.pc, p.prec) == (1.0, -1.0, 2, bt.PC_POLY, bt.F64)
    assert p.alpha[1] == 7.0 and p.max_outer == 30 and p.inner_tol == 1e-4


def test_struct_sizes_match_header(lib, tmp_path):
    """The ctypes mirror of bt_params and the numpy record of bt_info have
    the header's sizes and field offsets (the C compiler's, via gcc)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    fields = [f[0] for f in bt._Params._fields_]
    info = list(bt.INFO_DTYPE.names)
    src = tmp_path / "abi.c"
    src.write_text(
        "#include <stdio.h>\n#include <stddef.h>\n#include \"btpcg.h\"\n"
        "int main(void) {\n"
        '  printf("%zu\\n", sizeof(bt_params));\n' +
        "".join(f'  printf("%zu\\n", offsetof(bt_params, {f}));\n'
                for f in fields) +
        '  printf("%zu\\n", sizeof(bt_info));\n' +
        "".join(f'  printf("%zu\\n", offsetof(bt_info, {f}));\n'
                for f in info) +
        "  return 0;\n}\n")
    exe = str(tmp_path / "abi")
    subprocess.run([gcc, "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    exe], check=True)
    got = [int(v) for v in subprocess.run([exe], capture_output=True,
                                          text=True, check=True).stdout.split()]
    want = [ctypes.sizeof(bt._Params)] + \
        [getattr(bt._Params, f).offset for f in fields] + \
        [bt.INFO_DTYPE.itemsize] + [bt.INFO_DTYPE.fields[f][1] for f in info]
    assert got == want


def _ws(lib, B, off, n, params):
    off = np.asarray(off, dtype=np.int64)
    return lib.bt_workspace_bytes(B, off.ctypes.data_as(ctypes.c_void_p), n,
                                  ctypes.byref(params.to_c()))


def test_workspace_bytes_validation(lib):
    P = bt.Params.polycoeff(2)
    assert _ws(lib, 1, [0, 8], 4, P) > 0
    assert _ws(lib, 2, [0, 8, 8], 4, P) == 0           # empty instance
    assert _ws(lib, 1, [1, 8], 4, P) == 0              # offsets[0] != 0
    assert _ws(lib, 1, [0, 8], 0, P) == 0              # n < 1
    assert _ws(lib, 1, [0, 8], 65, P) == 0             # n > 64
    assert _ws(lib, 1, [0, 8], 4, bt.Params(a=0.5, b=0.5)) == 0   # 2a+b != 1
    assert _ws(lib, 1, [0, 8], 4, bt.Params(a=-0.1)) == 0         # a < 0
    assert _ws(lib, 1, [0, 8], 4, bt.Params(a=1.2)) == 0          # b < -1
    assert _ws(lib, 1, [0, 8], 4, bt.Params(m=0)) == 0
    assert _ws(lib, 1, [0, 8], 4, bt.Params(m=9)) == 0
    assert _ws(lib, 1, [0, 8], 4, bt.Params(prec="f32_ir", inner_tol=1.5)) == 0
    assert _ws(lib, 1, [0, 8], 4, bt.Params(warm_start=True)) > 0
    bad = bt.Params().to_c()
    bad.warm_start = 2                                  # neither 0 nor 1
    off = np.asarray([0, 8], dtype=np.int64)
    assert lib.bt_workspace_bytes(1, off.ctypes.data_as(ctypes.c_void_p), 4,
                                  ctypes.byref(bad)) == 0
    # f32 factors take half the bytes of f64 ones
    w64 = _ws(lib, 1, [0, 1000], 12, bt.Params(prec="f64"))
    w32 = _ws(lib, 1, [0, 1000], 12, bt.Params(prec="f32"))
    assert 1.9 < w64 / w32 < 2.1
    # float32 + refinement at n = 12 adds the packed L^{-1} of the
    # register-resident kernel: 80 floats per block row
    wir = _ws(lib, 1, [0, 1000], 12, bt.Params(prec="f32_ir"))
    assert 0 <= wir - w32 - 1000 * 80 * 4 < 512


def test_setup_rejects_before_touching_memory(lib):
    """Invalid calls return BT_EINVAL/BT_ENOSPACE without dereferencing the
    (deliberately bogus) device pointers and without any HIP call."""
    bogus = ctypes.c_void_p(0x1000)
    h = ctypes.c_void_p()
    off = np.array([0, 8], dtype=np.int64)
    offp = off.ctypes.data_as(ctypes.c_void_p)
    good = bt.Params.polycoeff(2).to_c()
    bad = bt.Params(a=2.0, b=-3.0).to_c()
    rc = lib.bt_batch_setup(ctypes.byref(h), 1, offp, 4, bt.DT_F64, bogus,
                            bogus, ctypes.byref(bad), bogus, 1 << 30, None)
    assert rc == bt.EINVAL and not h.value
    rc = lib.bt_batch_setup(ctypes.byref(h), 1, offp, 4, bt.DT_F64, bogus,
                            bogus, ctypes.byref(good), bogus, 16, None)
    assert rc == bt.ENOSPACE and not h.value
    rc = lib.bt_batch_setup(ctypes.byref(h), 1, offp, 4, 7, bogus, bogus,
                            ctypes.byref(good), bogus, 1 << 30, None)
    assert rc == bt.EINVAL
    rc = lib.bt_batch_setup(ctypes.byref(h), 1, offp, 4, bt.DT_F64, None,
                            bogus, ctypes.byref(good), bogus, 1 << 30, None)
    assert rc == bt.EINVAL
    rc = lib.bt_setup(ctypes.byref(h), 0, 4, bt.DT_F64, bogus, bogus,
                      ctypes.byref(good), bogus, 1 << 30, None)
    assert rc == bt.EINVAL
    # a batch with a system too large for one workgroup of the solve kernel
    # (a single system of that size is allowed: bt_solve_grid spans the grid)
    big = np.array([0, 8, 8 + (1 << 20)], dtype=np.int64)
    rc = lib.bt_batch_setup(ctypes.byref(h), 2,
                            big.ctypes.data_as(ctypes.c_void_p), 48,
                            bt.DT_F64, bogus, bogus, ctypes.byref(good), bogus,
                            1 << 40, None)
    assert rc == bt.EINVAL
    for fn in ("bt_solve", "bt_solve_batched"):
        assert getattr(lib, fn)(None, bogus, bogus, 1e-10, 10, bogus,
                                None) == bt.EINVAL
    assert lib.bt_precondition(None, bogus, bogus, None) == bt.EINVAL
    assert lib.bt_solve_adjoint(None, bogus, bogus, bogus, None, None, 1e-10,
                                10, bogus, None) == bt.EINVAL
    assert lib.bt_refactor(None, None) == bt.EINVAL
    assert lib.bt_solve_grid(None, bogus, bogus, 1e-10, 10, bogus, bogus,
                             1 << 20, None) == bt.EINVAL
    assert lib.bt_grid_workspace_bytes(None) == 0
    assert lib.bt_solve_grid_noalloc(None, bogus, bogus, 1e-10, 10, bogus,
                                     None) == bt.EINVAL


def test_kernel_configs_listed(lib):
    cfgs = bt.kernel_configs()
    assert len(cfgs) >= 4
    precs = {c[3] for c in cfgs}
    assert precs == {bt.F64, bt.F32}
    for _, nt, s, _ in cfgs:
        assert nt % 64 == 0 and nt <= 1024 and s >= 0
    # the register-resident bin kernel variants (s == 0): float32, 3, 6 and
    # 12 entries per lane, i.e. 1024, 512 and 256 threads, listed last
    fast = [c for c in cfgs if c[2] == 0]
    assert [c[1] for c in fast] == [1024, 512, 256]
    assert all(c[3] == bt.F32 for c in fast)
    assert [c[0] for c in fast] == list(range(len(cfgs) - 3, len(cfgs)))


def test_product_path_has_no_cpu_fallback():
    """The binding never imports the oracle and needs a GPU."""
    src = open(os.path.join(ROOT, "paper_2503_15269_amd", "__init__.py")).read()
    assert "import oracle" not in src and "from oracle" not in src
    import torch
    if not torch.cuda.is_available():
        with pytest.raises(RuntimeError):
            bt.Handle(torch.zeros(2, 2, 2, dtype=torch.float64),
                      torch.zeros(1, 2, 2, dtype=torch.float64))
