"""GPU: the alternative radix plans of the pencil passes (variants 3..5 of the
autotuner) on every length that has one, along the contiguous and the strided
axes, against the FP64 oracle; and the autotuner's process-wide choice."""
import os

import numpy as np
import pytest

import oracle as O
from paper_2404_10221_amd import rsfde as R
from rsfde_workloads import FieldSpec, Instance, config, with_grid

from gpu_helpers import dev, empty, host, rel, say, solver_for, tight

pytestmark = pytest.mark.gpu

# every length with an alternative plan: 256, 384, 512, 768, 1024, 1536, 2048,
# 3072, 4096, each on axis 1 and on a strided axis
ALT_SHAPES = [
    (2, (127, 191)), (2, (191, 127)), (2, (255, 383)), (2, (383, 255)),
    (2, (511, 7)), (2, (7, 511)), (2, (767, 5)), (2, (5, 767)),
    (2, (1023, 3)), (2, (3, 1023)), (2, (1535, 3)), (2, (3, 1535)),
    (2, (2047, 3)), (2, (3, 2047)),
    (3, (127, 5, 255)), (3, (5, 511, 3)),
]
ALT_L = {256, 384, 512, 768, 1024, 1536, 2048, 3072, 4096}


def _inst(d, n, seed):
    rng = np.random.default_rng(seed)
    alpha = tuple(float(a) for a in rng.uniform(1.1, 1.9, d))
    kappa = tuple(float(k) for k in rng.uniform(0.2, 2.0, d))
    return Instance(name=f"plan{d}", d=d, n=tuple(n), alpha=alpha, kappa=kappa, T=1.0, M=4,
                    e=FieldSpec("sinprod_cos", (2.0, 1.0)),
                    f=FieldSpec("sine_modes", (), modes=4, amp=rng.standard_normal(4 ** d),
                                time_dependent=False),
                    psi=FieldSpec("zero", time_dependent=False), restart=20, rtol=1e-10)


class _Forced:
    """RSFDE_FORCE_VARIANT for the handles created inside the block."""

    def __init__(self, v):
        self.v = v

    def __enter__(self):
        self.old = os.environ.get("RSFDE_FORCE_VARIANT")
        os.environ["RSFDE_FORCE_VARIANT"] = str(self.v)

    def __exit__(self, *exc):
        if self.old is None:
            del os.environ["RSFDE_FORCE_VARIANT"]
        else:
            os.environ["RSFDE_FORCE_VARIANT"] = self.old


@pytest.mark.parametrize("v", [3, 4, 5])
@pytest.mark.parametrize("d,n", ALT_SHAPES, ids=["x".join(map(str, s[1])) for s in ALT_SHAPES])
def test_alternative_plans_against_oracle(d, n, v):
    inst = _inst(d, n, seed=11)
    P = O.OracleProblem(inst, ebar=1.8)
    rng = np.random.default_rng(12)
    x = rng.standard_normal(P.shape)
    e = 1.0 + rng.random(P.shape)
    with _Forced(v):
        S = solver_for(inst, ebar=(1.8, 1.8))
    try:
        for ax in range(d):
            L = 2 * (n[ax] + 1)
            for tr in (0, 1):
                if d == 1 and tr == 1:
                    continue
                code, radices = R.rsfde_get_pass_plan(S.h, 0, ax, R.RSFDE_FP64, tr)
                want = L | (1 << 16) if L in ALT_L else L
                assert code == want and int(np.prod(radices)) == L, (ax, tr, code, radices)
        say(f"[plan v{v}] d={d} n={n}")
        out = empty(x.size)
        R.rsfde_apply_A(S.h, 0, dev(e), dev(x), out)
        assert rel(host(out), P.apply_A(e, x).ravel()) < 1e-12
        R.rsfde_apply_prec(S.h, 0, dev(x), out)
        assert rel(host(out), P.apply_prec_inv(x).ravel()) < 1e-12
    finally:
        S.close()


@pytest.mark.parametrize("wl,n", [("C2", (1023, 7)), ("C2", (7, 511)), ("C3", (5, 255, 7))])
def test_alternative_plans_fp32_inner_solves(wl, n):
    """The FP32 kernels of the alternative plans inside the mixed form's inner
    solves, against the oracle solved to rounding level."""
    inst = with_grid(config(wl), n, M=2)
    ref = O.run(tight(inst))
    with _Forced(3):
        S = solver_for(inst, precision=R.RSFDE_MIXED)
    u = empty(inst.size)
    R.rsfde_eval_field(S.h, 0, R.WHICH_PSI, 0.0, u)
    status, st = R.rsfde_solve(S.h, inst.M, [u])
    d = rel(host(u), ref["u"])
    say(f"[plan fp32] {wl} n={n}: rel diff {d:.3e}, sweeps {st[0]['outer_sweeps']}")
    S.close()
    assert status == R.RSFDE_OK and d <= 1e-10


def test_autotuner_choice_is_shared_by_the_handles_of_a_process():
    """Two handles on the same problem run the same kernels (plan and tile), so
    their results agree bit for bit."""
    inst = with_grid(config("C2"), (255, 383), M=2)
    codes, sols = [], []
    for _ in range(2):
        S = solver_for(inst)
        codes.append([R.rsfde_get_pass_plan(S.h, 0, ax, R.RSFDE_FP64, tr)[0]
                      for ax in range(2) for tr in (0, 1)]
                     + [R.rsfde_get_pass_shape(S.h, 0, ax, R.RSFDE_FP64, tr)[1]
                        for ax in range(2) for tr in (0, 1)])
        u = empty(inst.size)
        R.rsfde_eval_field(S.h, 0, R.WHICH_PSI, 0.0, u)
        R.rsfde_solve(S.h, inst.M, [u])
        sols.append(host(u))
        S.close()
    say(f"[tuner] plan codes and tiles {codes[0]}")
    assert codes[0] == codes[1]
    assert np.array_equal(sols[0], sols[1])
