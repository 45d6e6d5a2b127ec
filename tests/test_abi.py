"""C-ABI checks that need no GPU: the library loads, exports every entry
point that include/mx.h declares, and rejects bad arguments on the host
before any device call."""
import ctypes as C
import math
import os
import re

import pytest

from paper_1907_13088_amd import mx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_entry_points():
    src = open(os.path.join(ROOT, "include", "mx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mx_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = mx.lib()
    names = declared_entry_points()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_header_and_binding_struct_sizes_agree(tmp_path):
    """The ctypes mirrors of mx_config, mx_step_stats and mx_profile have the
    size and field offsets a C compiler gives the header's structs."""
    import subprocess
    structs = {"mx_config": mx.CConfig, "mx_step_stats": mx.CStats, "mx_profile": mx.CProfile}
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "mx.h"', "int main(void) {"]
    for name, cls in structs.items():
        src.append(f'printf("%zu", sizeof({name}));')
        for f, _ in cls._fields_:
            src.append(f'printf(" %zu", offsetof({name}, {f}));')
        src.append('printf("\\n");')
    src.append("return 0; }")
    (tmp_path / "probe.c").write_text("\n".join(src))
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.check_call(["gcc", "-I", inc, "-o", str(tmp_path / "probe"), str(tmp_path / "probe.c")])
    out = subprocess.check_output([str(tmp_path / "probe")], text=True).split("\n")
    for line, (name, cls) in zip(out, structs.items()):
        want = [C.sizeof(cls)] + [getattr(cls, f).offset for f, _ in cls._fields_]
        assert [int(v) for v in line.split()] == want, name
    c = mx.make_config(2, (16, 16), 0.3)
    assert mx.validate(c) == 0


def _cfg(**kw):
    base = dict(ndim=2, n=(32, 32), dt=0.5 / math.sqrt(2))
    base.update(kw)
    return mx.make_config(**base)


@pytest.mark.parametrize("kw,code", [
    (dict(dt=1.0), mx.MX_ECFL),
    (dict(dt=-0.1), mx.MX_EINVAL),
    (dict(dt=float("nan")), mx.MX_EINVAL),
    (dict(ndim=4), mx.MX_EINVAL),
    (dict(n=(0, 4)), mx.MX_EINVAL),
    (dict(d=(1.0, -1.0)), mx.MX_EINVAL),
    (dict(blocks=5), mx.MX_EINVAL),
    (dict(sweeps=-1), mx.MX_EINVAL),
    (dict(tol=-1e-3), mx.MX_EINVAL),
    (dict(filter_passes=9), mx.MX_EINVAL),
    (dict(sweeps_per_pass=17), mx.MX_EINVAL),
    (dict(sweeps_per_pass=9, variant=1), mx.MX_EINVAL),
    (dict(variant=5), mx.MX_EINVAL),
    (dict(form=7), mx.MX_EINVAL),
    (dict(solver=2), mx.MX_EINVAL),
    (dict(solver=1, variant=1), mx.MX_EINVAL),
    (dict(solver=1, form=1), mx.MX_EINVAL),
    (dict(solver=1, lumped=True), mx.MX_EINVAL),
    (dict(ndim=3, n=(8, 8, 8), d=(1.0, 1.0, 0.5), dt=0.3 / math.sqrt(3), solver=1), mx.MX_EINVAL),
    (dict(ndim=3, n=(8, 8, 8), dt=0.5 / math.sqrt(3), solver=1, sweeps_per_pass=4), mx.MX_EINVAL),
    (dict(ndim=3, n=(8, 8, 8), dt=0.5 / math.sqrt(3), blocks=1), mx.MX_EINVAL),
    (dict(ndim=3, n=(8, 8, 8), dt=0.5 / math.sqrt(3), sweeps_per_pass=4), mx.MX_EINVAL),
    (dict(ndim=3, n=(8, 8, 8), dt=0.5 / math.sqrt(3), dtype="f64", sweeps_per_pass=3), mx.MX_EINVAL),
    (dict(ndim=3, n=(8, 8, 8), dt=0.99 / math.sqrt(2)), mx.MX_ECFL),
    (dict(n=(32768, 32768)), mx.MX_EINVAL),
    (dict(ndim=3, n=(65536, 65536, 2), dt=0.5 / math.sqrt(3)), mx.MX_EINVAL),
])
def test_validation_errors(kw, code):
    with pytest.raises(mx.MxError) as ei:
        mx.validate(_cfg(**kw))
    assert ei.value.code == code
    assert len(mx.lib().mx_last_error()) > 0


def test_cfl_limit_is_inclusive_and_anisotropic():
    d = (1.0, 0.5)
    dt_cfl = 1.0 / math.sqrt(1 / d[0] ** 2 + 1 / d[1] ** 2)
    assert mx.validate(_cfg(d=d, dt=dt_cfl)) == 0
    with pytest.raises(mx.MxError):
        mx.validate(_cfg(d=d, dt=dt_cfl * 1.001))


def test_3d_convergence_guarantee_warning():
    # non-cubic 3D cells with dt above min(d)/sqrt(2): Appendix C bound lost
    d = (0.4, 1.0, 1.0)
    dt_cfl = 1.0 / math.sqrt(sum(1 / x ** 2 for x in d))
    c = mx.make_config(3, (8, 8, 8), 0.999 * dt_cfl, d=d)
    w = mx.validate(c)
    assert w & mx.WARN_NOCONV_GUARANTEE == (1 if 0.999 * dt_cfl > 0.4 / math.sqrt(2) else 0)
    c2 = mx.make_config(3, (8, 8, 8), 0.5 / math.sqrt(3))
    assert mx.validate(c2) == 0


def test_workspace_size_and_null_workspace():
    c = _cfg(dtype="f64")
    nbytes = mx.workspace_size(c)
    assert nbytes >= 15 * 32 * 32 * 8
    h = C.c_void_p()
    rc = mx.lib().mx_init(C.byref(c), None, None, 0, C.byref(h))
    assert rc == mx.MX_EWORKSPACE and not h.value
    rc = mx.lib().mx_init(C.byref(c), None, C.c_void_p(4096), 16, C.byref(h))
    assert rc == mx.MX_EWORKSPACE
    # the Chebyshev solve double-buffers its increments: three arrays more
    cc = _cfg(dtype="f64", solver=mx.SOLVER_CHEBYSHEV)
    assert mx.workspace_size(cc) - nbytes == 3 * 32 * 32 * 8


def test_step_rejects_null_grid():
    assert mx.lib().mx_step(None, 1, None, None, None) == mx.MX_EINVAL
    assert mx.lib().mx_bind_fields(None, None, None) == mx.MX_EINVAL


def test_batch_calls_reject_null_batch():
    L = mx.lib()
    assert L.mx_batch_step(None, 1, 0) == mx.MX_EINVAL
    assert L.mx_batch_get_plan(None, None, None, None) == mx.MX_EINVAL
    assert L.mx_batch_get_schedule(None, 1, None, None, None, None) == mx.MX_EINVAL
    assert L.mx_batch_bind(None, 0, None, None) == mx.MX_EINVAL
