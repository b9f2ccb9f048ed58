"""The oracle's pin tests and the library's host-side CPU tests run again
against AddressSanitizer / UndefinedBehaviorSanitizer builds (CPU only):
out-of-bounds accesses, use after free and undefined arithmetic in the C
oracle and in the library's host code (mesh and sweep-order construction,
velocity grids, CST fit, RBF factorisation) end the child run with an
error."""
import os

import pytest

import _sanitize as SZ

BAD = ("ERROR: AddressSanitizer", "runtime error:")


def _check(res):
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert not any(b in out for b in BAD), out[-4000:]
    return out


@pytest.mark.slow
def test_oracle_pins_under_asan_ubsan(tmp_path):
    lib = SZ.build_oracle(str(tmp_path / "liboracle_asan.so"))
    files = sorted(f"tests/{f}" for f in os.listdir(os.path.join(SZ.ROOT, "tests"))
                   if f.startswith("test_oracle_") and f.endswith(".py"))
    # the grid-refinement and finite-difference convergence runs are left out
    # (minutes under the sanitizers; the same code paths run in the others)
    res = SZ.run_pytest([*files, "-k", "not second_order_exact_gradient_matches_fd and not grid_convergence_order"
                                       " and not accelerates_near_the_continuum"
                                       " and not near_continuum_iteration_converges"],
                        {"ORACLE_LIB": lib, "LD_PRELOAD": SZ.gcc_asan_runtime()})
    out = _check(res)
    assert "passed" in out
    env = {"ORACLE_LIB": lib, "LD_PRELOAD": SZ.gcc_asan_runtime()}
    assert SZ.loaded_in_child("import oracle; oracle.lib()", lib, env)


@pytest.mark.slow
def test_library_host_code_under_asan_ubsan(tmp_path):
    rt = SZ.clang_asan_runtime()
    if not rt or not os.path.exists(os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")):
        pytest.skip("no hipcc / clang sanitizer runtime")
    lib = SZ.build_library(str(tmp_path / "libdvm_asan.so"))
    res = SZ.run_pytest(["tests/test_abi.py", "tests/test_shape_host.py", "-m", "not gpu"],
                        {"DVM_LIB": lib, "LD_PRELOAD": rt})
    out = _check(res)
    assert "passed" in out
    env = {"DVM_LIB": lib, "LD_PRELOAD": rt}
    assert SZ.loaded_in_child("from paper_2501_00923_amd import dvm; dvm.lib()", lib, env)
