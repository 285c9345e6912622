"""Host checks of the request loops' stop test for the learned stationary iteration."""
import math

from paper_2608_29082_amd.serve import Progress


def _run(seq, **kw):
    """seq: relative residuals at round ends every 8 cycles; the cycle count of the first failure, or None."""
    p = Progress(**kw)
    for k, r in enumerate(seq):
        if p.failed(8 * (k + 1), r, 5):
            return 8 * (k + 1)
    return None


def test_converging_iteration_never_fails():
    assert _run([0.5 * 0.8 ** k for k in range(400)]) is None           # slow, steady
    assert _run([1.5, 1.2] + [0.9 * 0.95 ** k for k in range(300)]) is None   # early bump above ||f||


def test_divergence_and_stall_rules():
    assert _run([100.0 ** k for k in range(10)]) == 40                   # 1e8 > diverge_factor 1e6 at cycle 40
    assert _run([2.0] * 20) == 64                                        # never below ||f|| by cycle 64
    assert _run([1.0] * 20) == 64                                        # no progress at all (exactly ||f||)
    # below ||f||, then slowly growing: the best stops improving; fails 128 cycles after it
    seq = [0.5 ** k for k in range(1, 11)] + [0.5 ** 10 * 1.01 ** k for k in range(1, 40)]
    assert _run(seq) == 80 + 128
    assert _run([0.1] * 40) == 8 + 128                                   # stagnation
    assert Progress().failed(8, 0.1, 6)                                  # the solver's own divergence flag
    assert Progress().failed(8, math.nan, 5)


def test_rules_can_be_switched_off():
    assert _run([2.0] * 40, stall_cycles=0, window=0) is None
    assert _run([0.1] * 40, window=0) is None
