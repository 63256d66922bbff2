"""Host-side checks of the C ABI (no compute calls, no GPU needed): the HIP
library loads and exports every symbol declared in include/mgpbd.h, the
Python binding knows exactly those names, the struct layouts agree, and the
host-side topology rules reject bad input before any device work."""
import ctypes as C
import os
import re

import pytest

from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "mgpbd.h")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mgpbd_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_four_paper_calls():
    names = declared()
    for n in ["mgpbd_create", "mgpbd_setup", "mgpbd_step", "mgpbd_solve"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2505_13390_amd import binding
    lib = binding.lib()
    for n in declared():
        assert hasattr(lib, n), n


def test_binding_covers_the_header():
    from paper_2505_13390_amd import binding
    assert sorted(binding.EXPORTED) == declared()


def test_options_struct_layout_matches_defaults():
    from paper_2505_13390_amd import binding
    o = binding.mgpbd_default_options()
    assert o.theta == 0.1 and o.gs_sweeps == 20 and o.pre_sweeps == 2 and o.post_sweeps == 2
    assert o.lambda_min == 0.1 and o.coarse_max == 400 and o.power_iters == 30
    assert o.omega_relax == 0.1 and o.tol == 1e-6 and o.seed == 20250513
    assert o.reuse_interval == 20 and o.precision == 0 and o.lmax_scale == 1.05
    assert o.use_graph == 1 and o.check_every == 8 and o.profile_spmv == 0
    assert o.spmv_tile == 0 and o.spmv_lanes == 0
    assert o.matrix_free == 1
    assert o.smoother == 0
    assert o.n_cand == 1
    assert o.power_max == 500 and o.power_tol == 1e-2
    assert o.vcycle_tail == 0 and o.fuse_transfers == 0 and o.resetup_on_breakdown == 1


def test_null_arguments_rejected_without_device_work():
    from paper_2505_13390_amd import binding
    lib = binding.lib()
    assert lib.mgpbd_create(None, None, None, 1.0, None, None, None) == binding.E_INVALID_ARG
    h = C.c_void_p()
    assert lib.mgpbd_step(None, None, None, None, None, None, None, 1, None) == binding.E_INVALID_ARG
    assert lib.mgpbd_num_levels(None, None) == binding.E_INVALID_ARG
    assert lib.mgpbd_last_error(None) == b"null context"
    assert lib.mgpbd_apply(None, None, None) == binding.E_INVALID_ARG
    assert lib.mgpbd_get_qr(None, 0, None, None, None, None) == binding.E_INVALID_ARG


def test_binding_rejects_host_and_short_tensors_before_calling_the_library():
    """The C ABI takes bare device pointers, so the binding checks device,
    dtype, contiguity and length itself; here on host tensors (no GPU)."""
    torch = pytest.importorskip("torch")
    from paper_2505_13390_amd import binding
    with pytest.raises(TypeError):
        binding._dev(torch.zeros(4, dtype=torch.float64))
    with pytest.raises(TypeError):
        binding._vec(torch.zeros(4, dtype=torch.float64), torch.float64, 4, "x")
    with pytest.raises(TypeError):
        binding._dev([0.0, 1.0])


def test_struct_offsets_match_the_header(tmp_path):
    """Every field offset and size of the option and statistics structs as a C
    compiler lays them out from include/mgpbd.h, against the binding's ctypes
    structs."""
    import shutil
    import subprocess
    from paper_2505_13390_amd import binding
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"mgpbd_options": binding.Options, "mgpbd_step_stats": binding.StepStats,
               "mgpbd_solve_stats": binding.SolveStats, "mgpbd_mesh": binding.Mesh,
               "mgpbd_constraints": binding.Constraints, "mgpbd_csr": binding.Csr}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mgpbd.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe),
                           str(src)])
    got = dict(l.rsplit(" ", 1) for l in subprocess.check_output([str(exe)]).decode().split("\n")
               if l)
    for cname, py in structs.items():
        assert int(got["%s size" % cname]) == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(got["%s.%s" % (cname, f)]) == getattr(py, f).offset, (cname, f)
