"""The library's interference estimator (ci_predict_slowdown, the rule the
sensitivity-aware admission applies; Section 5.1) against measured pairs
it was not fitted on: duty-axis HBM profiles of the request kinds, taken
from the stressor alone, predict the slowdown of a triad and of a GEMV
beside a triad co-runner (two kernels on two queues, the co-runner's device
stamps covering the victim's window)."""
import argparse

import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(dev):
    from paper_2501_16909_amd import coloc
    c = coloc.Context(0)
    yield c
    c.close()


def test_library_estimator_on_held_out_pairs(ctx):
    import bench
    from paper_2501_16909_amd import coloc
    args = argparse.Namespace(reps=5, deadline_ms=200)
    prof = bench.library_profiles(bench.serve_profiles(ctx, args, axis="duty", res=("hbm",)),
                                  bench.serve_profiles(ctx, args, axis="duty", hbm_mix="read", res=("hbm",)))
    co = bench.estimator_victim(ctx, "triad", 8020)
    errors = {}
    for kind, seed in (("triad", 7020), ("gemv", 7010)):
        victim = bench.estimator_victim(ctx, kind, seed)
        measured, trials, _ = bench.measure_pair(ctx, victim, co, reps=7)
        predicted = coloc.predict_slowdown(prof, kind, ["triad"])
        errors[kind] = abs(predicted - measured) / measured
        print(f"{kind} beside a triad: measured {measured:.3f} (streams {[round(t, 3) for t in trials]}), "
              f"predicted {predicted:.3f}")
        assert measured > 1.2          # a real interference, not noise
    # Both pairs are HBM-bound.  The measurement itself moves between boxes:
    # in five full estimator runs the GEMV beside a triad measured 1.70-2.61
    # (+-21 % around its mean) and the triad beside a triad 1.64-1.94, while
    # the rule predicted 2.29-2.43 and 1.88-1.93.  The bound covers that
    # spread on top of the estimator's own error (mean 0.21 over nine pairs);
    # a rule that ignored the co-runner (1.0) or priced it far off the
    # victim's curve would still fail.  The rule's arithmetic is checked
    # exactly against the oracle on the CPU.
    assert max(errors.values()) < 0.5, errors
