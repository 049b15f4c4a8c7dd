"""rpa_chi0_noalloc (the FP64 chi0 of one point with a fixed device scratch, for callers
that cannot allocate) against rpa_chi0 on the same device inputs: to rounding (the FP64
parity bar, element by element and in the Frobenius norm), on two calls in a row, the
second with a smaller system; sizes beyond the fixed scratch are refused on the host."""
import sys

import numpy as np
import pytest

from paper_2505_06021_amd import inputs

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-test] {msg}", file=sys.stderr, flush=True)


def rel_rows(a, b):
    return float(np.max(np.abs(a - b).max(axis=1) / np.abs(b).max(axis=1)))


def run_pair(ctx, s, iq, om):
    import torch
    from paper_2505_06021_amd import rpa
    s.materialize_B()
    m = rpa._Marshal(s, device=True)
    out = torch.full((s.naux, s.naux), float("nan"), dtype=torch.complex128, device="cuda:0")
    ctx.chi0_noalloc(m, iq, om, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref = ctx.chi0(s, iq, om, device=True)
    return got, ref


def test_noalloc_equals_chi0_on_two_calls_second_smaller():
    from paper_2505_06021_amd import rpa
    big = inputs.make_system("na_big", (2, 2, 1), 5, 40, 300, 3, 71, is_complex=True, sigma=0.1)
    small = inputs.make_system("na_small", (1, 1, 1), 3, 9, 70, 2, 72, is_complex=True, sigma=0.2,
                               periodic=False)
    with rpa.Context(0) as ctx:
        for s, iq in ((big, 3), (small, 0)):
            say(f"noalloc {s.name} N={s.naux} M={s.M}")
            got, ref = run_pair(ctx, s, iq, s.omega[1])
            assert np.all(np.isfinite(got))
            assert rel_rows(got, ref) <= 1e-12
            assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
            assert np.abs(got - got.conj().T).max() == 0.0


def test_noalloc_refuses_what_the_scratch_cannot_hold():
    import torch
    from paper_2505_06021_amd import rpa
    say("noalloc size and argument errors")
    # 100 x 90000 = 9e6 contraction rows: their weights alone exceed the 64 MiB scratch,
    # so the call is refused on the host before any launch (B is a real device array of
    # the full size; its values do not matter)
    big = inputs.make_system("na_rows", (1, 1, 1), 100, 90000, 1, 2, 74, is_complex=True, sigma=0.2,
                             periodic=False)
    with rpa.Context(0) as ctx:
        Bdev = torch.zeros((1, 1, 100, 90000, 1), dtype=torch.complex128, device="cuda:0")
        mb = rpa._Marshal(big, device=True, explicit_B=Bdev)
        outb = torch.empty((1, 1), dtype=torch.complex128, device="cuda:0")
        with pytest.raises(rpa.RpaError) as e:
            ctx.chi0_noalloc(mb, 0, 0.5, outb)
        assert e.value.code == rpa.RPA_E_NOMEM
        s = inputs.make_system("na_err", (1, 1, 1), 2, 3, 8, 2, 73, is_complex=True, sigma=0.2,
                               periodic=False)
        s.materialize_B()
        m = rpa._Marshal(s, device=True)
        out = torch.empty((s.naux, s.naux), dtype=torch.complex128, device="cuda:0")
        m2 = rpa._Marshal(s, device=False)            # host arrays are not accepted
        with pytest.raises(rpa.RpaError) as e:
            ctx.chi0_noalloc(m2, 0, 0.5, out)
        assert e.value.code == rpa.RPA_E_ARG
        with pytest.raises(rpa.RpaError) as e:
            ctx.chi0_noalloc(m, 0, 0.5, out, prec=rpa.FP32)
        assert e.value.code == rpa.RPA_E_ARG
