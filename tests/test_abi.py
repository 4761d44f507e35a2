"""The C-ABI library loads, exports every function include/hpic.h declares, its
ctypes structs match the C layout, and host-side validation rejects bad
configurations (Eq. (22) Courant limit, FFT size) before touching a device."""
import ctypes
import os
import re
import subprocess

import pytest

from tests.conftest import ROOT, ensure_hip_lib

HEADER = os.path.join(ROOT, "include", "hpic.h")


@pytest.fixture(scope="module")
def hp():
    ensure_hip_lib()
    from paper_1502_01376_amd import hpic
    return hpic


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hp_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(hp):
    names = _declared()
    assert len(names) >= 20
    assert sorted(hp.ABI) == names
    L = hp.lib()
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", hp.LIBPATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (hp_\w+)", out))
    assert set(names) <= exported


def test_struct_layout_matches_c(hp, tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stddef.h>
#include <stdio.h>
#include "hpic.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(hp_config), offsetof(hp_config, dt),
         offsetof(hp_config, filter_frac), offsetof(hp_config, sort_interval),
         sizeof(hp_diag), offsetof(hp_diag, step));
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    C, D = hp.Config, hp.Diag
    want = [ctypes.sizeof(C), C.dt.offset, C.filter_frac.offset, C.sort_interval.offset,
            ctypes.sizeof(D), D.step.offset]
    assert got == want


def _create(hp, cfg):
    h = ctypes.c_void_p()
    arr = (hp.Config * 1)(cfg)
    rc = hp.lib().hp_create(arr, 1, ctypes.byref(h))
    if rc == 0:
        hp.lib().hp_destroy(h)
    return rc, hp.lib().hp_last_error().decode()


def test_courant_violation_rejected(hp):
    import oracle
    lim = oracle.courant_limit2(0.1, 0.2)
    rc, msg = _create(hp, hp.config(64, 32, 0.1, 0.2, lim * 1.001))
    assert rc == hp.HP_ECOURANT, msg
    # the finite-difference (Yee) mode has the larger Yee limit
    rc, _ = _create(hp, hp.config(64, 32, 0.1, 0.2, lim * 1.001, deriv1=1))
    assert rc != hp.HP_ECOURANT


@pytest.mark.parametrize("n1,n2,prec", [(48, 32, "fp32"), (4, 32, "fp32"), (16384, 8, "fp32"),
                                        (16384, 8, "fp64"), (64, 3, "fp32")])
def test_bad_grid_rejected(hp, n1, n2, prec):
    rc, msg = _create(hp, hp.config(n1, n2, 0.2, 0.2, 0.05, precision=prec))
    assert rc == hp.HP_EINVAL, msg


def test_q3d_n1_limit(hp):
    rc, msg = _create(hp, hp.config(8192, 16, 0.2, 0.2, 0.05, modes=2))
    assert rc == hp.HP_EINVAL, msg


def test_bad_precision_and_shape_rejected(hp):
    c = hp.config(64, 32, 0.2, 0.2, 0.05)
    c.precision = 7
    assert _create(hp, c)[0] == hp.HP_EINVAL
    c = hp.config(64, 32, 0.2, 0.2, 0.05)
    c.shape_order = 4
    assert _create(hp, c)[0] == hp.HP_EINVAL
    c = hp.config(32, 16, 0.2, 0.2, 0.02, n3=16, dx3=0.2)  # cubic is 2D only
    c.shape_order = 3
    assert _create(hp, c)[0] == hp.HP_EINVAL
    c = hp.config(64, 32, 0.2, 0.2, 0.05)
    c.interp = 2
    assert _create(hp, c)[0] == hp.HP_EINVAL


def test_no_cpu_fallback_without_device(hp):
    """Without a GPU the library reports HP_EDEVICE; it never computes on the host."""
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    if has_gpu:
        pytest.skip("a GPU is present")
    rc, msg = _create(hp, hp.config(64, 32, 0.2, 0.2, 0.05))
    assert rc == hp.HP_EDEVICE, msg
