"""Host-side checks of the C ABI: the library loads, exports every entry point
that include/ulppm.h declares, and the ctypes mirrors of the structs match the
header's layout (sizes and offsets measured by compiling the header with gcc).
No GPU call is made."""
import os
import re
import subprocess
import tempfile

import pytest

from paper_2203_05562_amd import ulppm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ulppm.h")


def declared_symbols():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(ulppm_\w+)\s*\(", txt, re.M)))


def test_header_declares_expected_entry_points():
    syms = declared_symbols()
    for s in ("ulppm_build_families", "ulppm_step", "ulppm_forces", "ulppm_create", "ulppm_destroy"):
        assert s in syms
    assert set(syms) == set(ulppm.EXPORTS)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ulppm.LIB_PATH):
        from paper_2203_05562_amd.build import build
        build()
    return ulppm.load_library()


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", ulppm.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r" T (ulppm_\w+)", out))
    missing = [s for s in declared_symbols() if s not in exported]
    assert not missing, missing
    for s in declared_symbols():
        assert hasattr(lib, s)


def test_struct_layout_matches_header():
    prog = r'''
#include <stdio.h>
#include <stddef.h>
#include "ulppm.h"
int main(void) {
  printf("%zu %zu %zu\n", sizeof(ulppm_params), sizeof(ulppm_state), sizeof(ulppm_report));
  printf("%zu %zu %zu %zu\n", offsetof(ulppm_params, g), offsetof(ulppm_params, newton_maxit),
         offsetof(ulppm_params, energy_tol), offsetof(ulppm_state, sig));
  printf("%zu %zu %zu %zu\n", offsetof(ulppm_state, fixed), offsetof(ulppm_report, steps),
         offsetof(ulppm_params, timing), offsetof(ulppm_report, t_gather_ms));
  printf("%zu %zu\n", offsetof(ulppm_report, t_kin_ms), offsetof(ulppm_report, n_rebuilds));
  printf("%zu %zu %zu\n", sizeof(ulppm_contact), offsetof(ulppm_contact, spacing), offsetof(ulppm_contact, n));
  return 0;
}
'''
    import ctypes as C
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(src, "w").write(prog)
        subprocess.run(["gcc", "-I", os.path.dirname(HEADER), "-o", exe, src], check=True)
        vals = [int(v) for v in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()]
    exp = [C.sizeof(ulppm.Params), C.sizeof(ulppm.State), C.sizeof(ulppm.Report),
           ulppm.Params.g.offset, ulppm.Params.newton_maxit.offset, ulppm.Params.energy_tol.offset,
           ulppm.State.sig.offset, ulppm.State.fixed.offset, ulppm.Report.steps.offset,
           ulppm.Params.timing.offset, ulppm.Report.t_gather_ms.offset, ulppm.Report.t_kin_ms.offset,
           ulppm.Report.n_rebuilds.offset, C.sizeof(ulppm.Contact), ulppm.Contact.spacing.offset, ulppm.Contact.n.offset]
    assert vals == exp


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(ImportError):
        saved = ulppm._lib
        ulppm._lib = None
        try:
            ulppm.load_library(str(tmp_path / "nope.so"))
        finally:
            ulppm._lib = saved


def test_tail_adjoint_selfcheck_on_host(lib):
    """The library's hand-written reverse of the per-bond tail (inversion,
    velocity gradient, strain increment, Perzyna return map through the
    implicit-function theorem, force-state factor) agrees with central
    differences on the host, elastic and plastic bonds alike."""
    from paper_2203_05562_amd import inputs
    prm = ulppm.make_params(inputs.default_params(inputs.CONFIGS["C0"], 20e3), dt=2.8e-5)
    for seed in range(4):
        err, npl = ulppm.selfcheck_tail(prm, seed, 40)
        assert npl == 20
        assert err < 2e-5, (seed, err)
