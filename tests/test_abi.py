"""The C ABI library loads, exports every function include/mgdamg.h declares,
and its struct layouts match the Python binding (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mgdamg.h")


def _header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\*?\s+\*?([a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2002_04958_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2002_04958_amd import build
        build.build(verbose=False)
    return _lib.load()


def test_header_declares_the_boundary():
    names = _header_functions()
    for required in ("amg_setup", "block_precond_create", "gmres_solve", "adjoint_solve"):
        assert required in names
    assert len(names) >= 30


def test_every_declared_symbol_is_exported(lib):
    from paper_2002_04958_amd import _lib
    names = _header_functions()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    bound = sorted(n for n, _, _ in _lib.SIGNATURES)
    assert bound == names


def test_host_defaults_follow_the_paper(lib):
    from paper_2002_04958_amd import _lib
    p = _lib.amg_params()
    lib.amg_params_default(ctypes.byref(p))
    assert p.strength_theta == 0.25 and p.coarse_max == 100 and p.n_pre == 1 and p.n_post == 1
    assert p.dominance_theta == 0.9 and p.max_levels == 25 and p.aggressive_levels == 0
    g = _lib.gmres_params()
    lib.gmres_params_default(ctypes.byref(g))
    assert g.restart == 30 and g.rtol == 1e-8 and g.max_iters == 1000
    b = _lib.block_params()
    lib.block_params_default(ctypes.byref(b))
    assert b.kind == _lib.PC_KINDS["schur2"] and b.pctl_p_tol == 1e-2
    assert b.adaptive == 0 and b.theta_wc == 1e-2 and b.sigma_wc == 0.5
    assert b.theta_wd == 0.9 and b.jacobi_sweeps == 2
    assert b.inner_tol == 0.0 and b.inner_maxcycles == 100 and b.option4_steps == 0
    assert lib.mgd_kernel_class_count() >= 8
    assert lib.mgd_kernel_class_name(0) == b"spmv"
    assert b"gfx950" in lib.mgd_version()


def test_struct_layouts_match_c(tmp_path):
    from paper_2002_04958_amd import _lib
    structs = ["mgd_csr", "amg_params", "amg_info", "mgd_block_system", "mgd_coeffs",
               "block_params", "block_precond_info", "gmres_params", "gmres_result",
               "mgd_allocator"]
    src = "#include <stdio.h>\n#include <stddef.h>\n#include \"mgdamg.h\"\nint main(void){\n"
    for s in structs:
        src += f'  printf("{s} %zu\\n", sizeof({s}));\n'
    src += '  printf("block_params.pctl_p_tol %zu\\n", offsetof(block_params, pctl_p_tol));\n'
    src += '  printf("gmres_result.relres_est %zu\\n", offsetof(gmres_result, relres_est));\n'
    src += '  printf("block_params.jacobi_sweeps %zu\\n", offsetof(block_params, jacobi_sweeps));\n'
    src += '  printf("block_precond_info.jacobi %zu\\n", offsetof(block_precond_info, jacobi));\n'
    src += '  printf("block_params.inner_maxcycles %zu\\n", offsetof(block_params, inner_maxcycles));\n'
    src += '  printf("block_params.option4_steps %zu\\n", offsetof(block_params, option4_steps));\n'
    src += '  printf("block_precond_info.inner_cycles %zu\\n", offsetof(block_precond_info, inner_cycles));\n'
    src += '  printf("amg_params.aggressive_levels %zu\\n", offsetof(amg_params, aggressive_levels));\n'
    src += "  return 0;\n}\n"
    c = tmp_path / "probe.c"
    c.write_text(src)
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    got = dict(line.split() for line in out.strip().splitlines())
    for s in structs:
        assert int(got[s]) == ctypes.sizeof(getattr(_lib, s)), s
    assert int(got["block_params.pctl_p_tol"]) == _lib.block_params.pctl_p_tol.offset
    assert int(got["gmres_result.relres_est"]) == _lib.gmres_result.relres_est.offset
    assert int(got["block_params.jacobi_sweeps"]) == _lib.block_params.jacobi_sweeps.offset
    assert int(got["block_precond_info.jacobi"]) == _lib.block_precond_info.jacobi.offset
    assert int(got["block_params.inner_maxcycles"]) == _lib.block_params.inner_maxcycles.offset
    assert int(got["block_params.option4_steps"]) == _lib.block_params.option4_steps.offset
    assert int(got["block_precond_info.inner_cycles"]) == _lib.block_precond_info.inner_cycles.offset
    assert int(got["amg_params.aggressive_levels"]) == _lib.amg_params.aggressive_levels.offset


def test_product_path_has_no_cpu_fallback():
    """The package fails loudly without the library and never imports the oracle."""
    import paper_2002_04958_amd
    from paper_2002_04958_amd import _lib
    pkg = os.path.dirname(paper_2002_04958_amd.__file__)
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            text = open(os.path.join(pkg, fn)).read()
            assert "import oracle" not in text and "from oracle" not in text, fn
    with pytest.raises(_lib.LibraryMissing):
        saved = _lib._LIB
        _lib._LIB = None
        try:
            _lib.load(os.path.join(pkg, "does_not_exist.so"))
        finally:
            _lib._LIB = saved
