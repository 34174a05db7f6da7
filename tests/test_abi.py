"""CPU checks of the C ABI library: it builds for gfx950, loads, and exports every
function that include/ulisse_gp.h declares.  No compute call is made (no GPU here)."""
import ctypes
import os
import subprocess

import pytest

from paper_1501_05427_amd import binding, build


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        build.build()
    return binding.lib()


def test_header_declares_the_boundary():
    names = binding.header_functions()
    for f in ["gp_create", "gp_destroy", "gp_last_error", "gp_kmv", "gp_dkmv", "ulisse_solve",
              "gp_stoch_grad", "sgld_step", "gp_draw_probes", "gp_philox", "gp_profile",
              "gp_profile_read"]:
        assert f in names, f


def test_every_declared_symbol_is_exported(lib):
    for name in binding.header_functions():
        assert hasattr(lib, name), name


def test_struct_layouts_match_the_header(tmp_path):
    # the C compiler's view of the structs (size and every field offset) vs ctypes
    structs = {"gp_data": binding.gp_data, "ulisse_params": binding.ulisse_params,
               "ulisse_sysstat": binding.ulisse_sysstat, "gp_prior": binding.gp_prior,
               "gp_profile_stats": binding.gp_profile_stats, "gp_precond": binding.gp_precond,
               "gp_shift_precond": binding.gp_shift_precond, "sgld_schedule": binding.sgld_schedule,
               "sgld_state": binding.sgld_state, "gp_batch_problem": binding.gp_batch_problem,
               "gp_batch_stats": binding.gp_batch_stats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ulisse_gp.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    inc = os.path.dirname(binding.HEADER)
    subprocess.run(["gcc", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                 check=True).stdout.splitlines())
    for cname, cls in structs.items():
        assert int(out[cname]) == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert int(out[f"{cname}.{fname}"]) == getattr(cls, fname).offset, (cname, fname)


def test_constants_match_the_header():
    # the statistics flags, precision codes and status codes the binding uses, against the
    # header's #defines and enumerators
    import re
    text = open(binding.HEADER).read()
    defines = {k: int(v) for k, v in re.findall(r"#define\s+(ULISSE_\w+)\s+(\d+)u", text)}
    assert defines == {"ULISSE_NOTCONV": 1, "ULISSE_BREAKDOWN": 2, "ULISSE_FALLBACK": 4, "ULISSE_FP32_RERUN": 8}
    for k, v in defines.items():
        assert getattr(binding, k) == v, k
    for k in ("GP_FP32", "GP_BF16_SPLIT_V", "GP_BF16_SPLIT_KV", "GP_OK", "GP_EINVAL", "GP_ENOMEM",
              "GP_EDEVICE", "GP_EUNSUPPORTED"):
        m = re.search(rf"\b{k}\s*=\s*(-?\d+)", text)
        assert m is not None and int(m.group(1)) == getattr(binding, k), k


def test_validation_is_synchronous_and_host_side(lib):
    # bad sizes are rejected before any device work: the null handle is caught first
    st = lib.gp_kmv(None, binding.gp_data(0, 0, 0, 0), None, None, 0, 0, None, 0, 0, None)
    assert st == binding.GP_EINVAL
    assert b"handle" in lib.gp_last_error()
    st = lib.gp_philox(0, 0, 0, 0, 0, 0, -1, None, None)
    assert st == binding.GP_EINVAL
    # the shifted preconditioner, the autotuner and the batch validate before device work too
    p = binding.make_params()
    sp = binding.make_shift_precond(0.1)
    st = lib.ulisse_solve_shift_pc(None, binding.gp_data(0, 0, 0, 0), None, None, 1, 1, None,
                                   ctypes.byref(p), ctypes.byref(sp), None, None, None, None)
    assert st == binding.GP_EINVAL
    assert lib.gp_autotune(None, 1) == binding.GP_EINVAL
    code, split = ctypes.c_int32(0), ctypes.c_int32(0)
    assert lib.gp_tune_set(None, 4096, 4, 16, 0, 0) == binding.GP_EINVAL
    assert lib.gp_tune_get(None, 4096, 4, 16, 0, ctypes.byref(code), ctypes.byref(split)) == binding.GP_EINVAL
    assert lib.gp_tune_save(None, b"/nonexistent/x") == binding.GP_EINVAL
    assert lib.gp_tune_load(None, b"/nonexistent/x") == binding.GP_EINVAL
    out = ctypes.c_void_p()
    descs = (binding.gp_batch_problem * 1)()
    st = lib.gp_batch_create(ctypes.byref(out), 0, 0, 0, descs, 4, 0, 20, ctypes.byref(p), 8, 0, 1)
    assert st == binding.GP_EINVAL and out.value is None           # B = 0
    st = lib.gp_batch_create(ctypes.byref(out), 0, 0, 1, descs, 4, 0, 20, ctypes.byref(p), 7, 0, 1)
    assert st == binding.GP_EINVAL and b"iters_per_graph" in lib.gp_last_error()
    st = lib.gp_batch_create(ctypes.byref(out), 0, 0, 1, descs, 4, 0, 20, ctypes.byref(p), 8, 0, 1)
    assert st == binding.GP_EINVAL                                  # problem 0 has no X


def test_sources_are_gfx950_only():
    src = open(os.path.join(binding.HERE, "build.py")).read()
    assert "--offload-arch={ARCH}" in src and 'ARCH = "gfx950"' in src
    assert "-packed-fp32-ops" in src
