"""The C ABI library loads and exports every symbol include/ma_ot.h declares (no GPU calls)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ma_ot.h")
LIB = os.path.join(ROOT, "paper_1009_6039_amd", "libmaot.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ma3?_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libmaot.so is not built (python -m paper_1009_6039_amd.build)")
    return ctypes.CDLL(LIB)


def test_header_declares_the_expected_entry_points():
    names = declared_functions()
    for must in ("ma_plan_create", "ma_plan_destroy", "ma_solve", "ma_solve_batched",
                 "ma_step_residual", "ma_step_strain_apply", "ma_step_gmres"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_1009_6039_amd import maot
    assert sorted(maot.EXPORTED) == declared_functions()


def test_abi_version_matches_header(lib):
    m = re.search(r"#define MA_OT_ABI_VERSION (\d+)", open(HEADER).read())
    assert lib.ma_abi_version() == int(m.group(1))


def test_default_options_and_error_strings(lib):
    from paper_1009_6039_amd import maot
    o = maot.make_options()
    assert (o.max_newton, o.gmres_m, o.gmres_max_restarts) == (100, 10, 20)
    assert o.gmres_tol == 1e-4 and o.max_backtrack == 12 and o.wait_limit_s == 600.0
    # the linear step of Section 4.2 by default; BiCG capped at 1000 iterations (Section 5.1)
    assert o.linear_solver == maot.LINEAR["strain_gmres"] and o.bicg_max_iters == 1000
    assert maot.strerror(0) == "converged"
    assert "invalid" in maot.strerror(-1)


@pytest.mark.parametrize("n", [0, 8, 15, 24, 40, 4096])
def test_plan_create_rejects_unsupported_sizes_without_touching_the_gpu(lib, n):
    from paper_1009_6039_amd import maot
    h = ctypes.c_void_p()
    o = maot.make_options()
    assert lib.ma_plan_create(n, 1, ctypes.byref(o), ctypes.byref(h)) == -1
    assert h.value is None


def test_plan_create_rejects_bad_options(lib):
    from paper_1009_6039_amd import maot
    h = ctypes.c_void_p()
    for bad in (dict(gmres_m=0), dict(gmres_m=31), dict(gmres_tol=0.0), dict(interp=7),
                dict(damping_policy=3), dict(max_backtrack=-1), dict(wait_limit_s=0.0),
                dict(wait_limit_s=-1.0), dict(linear_solver=2), dict(linear_solver="fd_bicg", bicg_max_iters=0),
                dict(linear_solver="fd_bicg", precond="diag")):
        o = maot.make_options(**bad)
        assert lib.ma_plan_create(64, 1, ctypes.byref(o), ctypes.byref(h)) == -1


SIZES = (16, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048)


@pytest.mark.parametrize("n", SIZES)
def test_tune_geometry_table_is_consistent(n):
    # every variant of every kernel class tiles the grid exactly with whole
    # wavefronts; duplicates point at a smaller index with the same geometry.
    # Variants 0..3 are the block-shared kernels, 4 and 5 the wave-owned ones, 6, 7
    # of row pass C the block-shared ones that load coefficients first, and 8..11 the
    # radix plans (8, 10 one plan, 9, 11 the other): a geometry is distinct within its
    # family.
    from paper_1009_6039_amd import maot
    for k in maot.TUNE_PASSES:
        seen = {}
        for v in range(maot.TUNE_VARIANTS):
            canon, units, threads = maot.tune_geometry(k, n, v)
            assert 0 <= canon <= v and units >= 1 and threads % 64 == 0 and 64 <= threads <= 1024
            if k in ("row_a", "row_c"):
                assert (n // 2) % units == 0
            elif k == "column":
                assert (n // 2) % units == 0 and (n * units) % threads == 0 and threads % units == 0
            else:
                assert n % units == 0 and units >= 16
            if canon < 8:
                family = 0 if canon < 4 else (1 if canon < 6 else 2)
            else:
                family = 3 + canon % 2
            if canon < v:
                assert seen[canon][1:] == (units, threads)
            else:
                assert (family, units, threads) not in seen.values()
            seen[v] = (family, units, threads)


def test_tune_geometry_rejects_bad_arguments():
    from paper_1009_6039_amd import maot
    assert maot.tune_geometry("row_c", 500, 0)[0] == -1
    assert maot.tune_geometry("row_c", 512, maot.TUNE_VARIANTS)[0] == -1
    assert maot.tune_geometry("row_c", 512, -1)[0] == -1
    assert maot.tune_geometry(7, 512, 0)[0] == -1


def test_bench_refuses_several_gpus():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_pass_kernel_names_follow_the_variant_table():
    # the names the profilers print for the kernels a variant launches (used to match
    # rocprofv3 summaries to the tuned geometry)
    from paper_1009_6039_amd import maot
    assert maot.pass_kernel_name("row_c", 512, 3) == "k_passC<512, 3, false, 0>"
    assert maot.pass_kernel_name("row_c", 512, 1) == "k_passC<512, 0, false, 0>"  # a duplicate of 0
    assert maot.pass_kernel_name("row_c", 512, 7) == "k_passC<512, 3, true, 0>"
    assert maot.pass_kernel_name("row_c", 512, 4) == "k_passC_w<512, 1>"
    assert maot.pass_kernel_name("row_c", 384, 11) == "k_passC<384, 3, false, 2>"
    assert maot.pass_kernel_name("row_a", 512, 2) == "k_passA<512, 2, 0>"
    assert maot.pass_kernel_name("column", 1024, 9) == "k_passB<1024, 0, 2>"
    assert maot.pass_kernel_name("residual", 512, 3) is None
    assert maot.pass_kernel_name("row_c", 500, 0) is None
