"""Host-side checks of the C ABI: the library loads and exports every symbol the
header declares, and argument validation answers before any HIP call (these
tests run on machines without a GPU)."""
import os
import re

import pytest

from paper_2404_10221_amd import rsfde as R
from rsfde_workloads import config, paper_example

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rsfde.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(rsfde_\w+)\s*\(", txt, re.M)))


def test_library_exports_every_declared_symbol():
    lib = R.load_library()
    names = _declared()
    assert len(names) >= 16
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(R.EXPORTED)


def test_workspace_sizes_of_the_workloads():
    for name in ("C1", "C2", "C3", "C5"):
        inst = config(name)
        b = R.rsfde_workspace_size([R.params_from_instance(inst)])
        # at least (restart + 8) FP64 vectors
        assert b >= (inst.restart + 8) * inst.size * 8
    c4 = config("C4")
    assert len(c4) == 64
    b = R.rsfde_workspace_size([R.params_from_instance(i) for i in c4])
    assert b > sum((i.restart + 8) * i.size * 8 for i in c4)


def _base(**over):
    kw = dict(d=2, n=(15, 23), alpha=(1.3, 1.7), kappa=(1.0, 0.5), dt=0.01)
    kw.update(over)
    d = kw.pop("d")
    return R.make_params(d, kw.pop("n"), kw.pop("alpha"), kw.pop("kappa"), kw.pop("dt"), **kw)


@pytest.mark.parametrize("over,code", [
    (dict(d=0), R.RSFDE_E_INVALID_ARG),
    (dict(d=4, n=(15, 15, 15), alpha=(1.5,) * 3, kappa=(1,) * 3), R.RSFDE_E_INVALID_ARG),
    (dict(n=(0, 15)), R.RSFDE_E_INVALID_ARG),
    (dict(alpha=(1.0, 1.5)), R.RSFDE_E_INVALID_ARG),
    (dict(alpha=(1.5, 2.0)), R.RSFDE_E_INVALID_ARG),
    (dict(kappa=(-1.0, 1.0)), R.RSFDE_E_INVALID_ARG),
    (dict(kappa=(0.0, 0.0)), R.RSFDE_E_INVALID_ARG),
    (dict(dt=0.0), R.RSFDE_E_INVALID_ARG),
    (dict(e_min=-1.0, e_max=2.0), R.RSFDE_E_INVALID_ARG),
    (dict(e_min=3.0, e_max=2.0), R.RSFDE_E_INVALID_ARG),
    (dict(restart=0), R.RSFDE_E_INVALID_ARG),
    (dict(restart=65), R.RSFDE_E_INVALID_ARG),
    (dict(rtol=0.0), R.RSFDE_E_INVALID_ARG),
    (dict(max_cycles=0), R.RSFDE_E_INVALID_ARG),
    (dict(precision=2), R.RSFDE_E_INVALID_ARG),
    (dict(x0_mode=3), R.RSFDE_E_INVALID_ARG),
    (dict(method=3), R.RSFDE_E_INVALID_ARG),
    (dict(precision=R.RSFDE_MIXED, rtol=1e-10, outer_rtol=1e-9), R.RSFDE_E_INVALID_ARG),
    (dict(precision=R.RSFDE_MIXED, outer_rtol=-1e-12), R.RSFDE_E_INVALID_ARG),
    (dict(method=R.RSFDE_SPGM, precision=R.RSFDE_MIXED), R.RSFDE_E_UNSUPPORTED),
    (dict(method=R.RSFDE_TPGM, precision=R.RSFDE_MIXED), R.RSFDE_E_UNSUPPORTED),
    (dict(lo=(0.0, 1.0), hi=(1.0, 1.0)), R.RSFDE_E_INVALID_ARG),
    (dict(n=(14, 15)), R.RSFDE_E_UNSUPPORTED),      # 2(N+1) = 30 is not 2^p or 3*2^p
    (dict(n=(4095, 15)), R.RSFDE_E_UNSUPPORTED),    # 2(N+1) = 8192 > 4096
])
def test_validation_errors_before_any_device_call(over, code):
    with pytest.raises(R.RsfdeError) as ei:
        R.rsfde_workspace_size([_base(**over)])
    assert ei.value.status == code


def test_supported_sizes_validate():
    for n in (3, 5, 7, 11, 15, 23, 31, 47, 63, 95, 127, 191, 255, 383, 511, 767, 1023, 1535, 2047):
        R.rsfde_workspace_size([_base(n=(n, 7))])


def test_setup_rejects_small_or_missing_workspace_without_touching_the_device():
    import ctypes as C
    p = _base()
    arr = (R.rsfde_params * 1)(p)
    h = C.c_void_p()
    lib = R.load_library()
    assert lib.rsfde_setup(arr, 1, None, 0, None, C.byref(h)) == R.RSFDE_E_WORKSPACE
    buf = (C.c_char * 1024)()
    assert lib.rsfde_setup(arr, 1, C.addressof(buf), 1024, None, C.byref(h)) == R.RSFDE_E_WORKSPACE
    assert lib.rsfde_setup(arr, 0, None, 0, None, C.byref(h)) == R.RSFDE_E_INVALID_ARG
    assert lib.rsfde_setup(None, 1, None, 0, None, C.byref(h)) == R.RSFDE_E_INVALID_ARG


def test_strerror_texts():
    for s in (0, 1, -1, -2, -3, -4, -5, -6):
        assert len(R.strerror(s)) > 0
    assert "unknown" in R.strerror(-99)


def test_null_handle_calls_fail_cleanly():
    lib = R.load_library()
    assert lib.rsfde_destroy(None) == R.RSFDE_E_INVALID_ARG
    assert lib.rsfde_set_ebar(None, 0, 1.0, 2.0) == R.RSFDE_E_INVALID_ARG
    assert lib.rsfde_apply_A(None, 0, None, None, None) == R.RSFDE_E_INVALID_ARG
    assert lib.rsfde_set_timing(None, 1, 1) == R.RSFDE_E_INVALID_ARG
    assert lib.rsfde_set_graph(None, 1) == R.RSFDE_E_INVALID_ARG
    assert lib.rsfde_set_true_residual(None, 1) == R.RSFDE_E_INVALID_ARG
    assert lib.rsfde_apply_prec_form(None, 0, 1, None, None) == R.RSFDE_E_INVALID_ARG
    assert lib.rsfde_get_pass_shape(None, 0, 0, 0, 0, None, None) == R.RSFDE_E_INVALID_ARG
    assert lib.rsfde_solve(None, 1, R.SAMPLE_FN(0), None, None, None) == R.RSFDE_E_INVALID_ARG
    assert lib.rsfde_solve_range(None, 0, 1, R.SAMPLE_FN(0), None, None, None) == R.RSFDE_E_INVALID_ARG


def test_params_from_paper_example():
    p = R.params_from_instance(paper_example(2, (1.1, 1.3), 16, 4096))
    assert p.d == 2 and p.n[0] == 15 and abs(p.dt - 1 / 4096) < 1e-18
    assert R.rsfde_workspace_size([p]) > 0


def test_shipped_tune_cache_is_well_formed():
    """tune_cache.txt beside the library: comment lines, then one
    'arch d<d> ax<a> fp<p> cls<c> L<len>=<variant>' line per autotuned pass, each
    key once, variants 0..5, and only transform lengths the library carries."""
    import os
    import re
    path = os.path.join(os.path.dirname(R.__file__), "tune_cache.txt")
    assert os.path.exists(path)
    seen = set()
    pat = re.compile(r"^(gfx\S+) d([123]) ax([012]) fp([01]) cls([01]) L(\d+)=([0-5])$")
    lengths = {8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048,
               3072, 4096}
    for line in open(path).read().splitlines():
        if not line or line.startswith("#"):
            assert "=" not in line  # the loader would read it as an entry
            continue
        m = pat.match(line)
        assert m, line
        key = line.rsplit("=", 1)[0]
        assert key not in seen, key
        seen.add(key)
        d, ax = int(m.group(2)), int(m.group(3))
        assert ax < d and int(m.group(6)) in lengths, line
    assert len(seen) >= 30
