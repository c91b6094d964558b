"""The training schedule's stage decisions (Sec. 4.3: a warm-up of up to 500
iterations, then densification and static identification every 100
iterations, densifying up to iteration 15,000 as in Sec. 5.2), and the
densification limits as the library receives them (no GPU)."""
import math

from paper_2505_13215_amd.train import DensifyLimits, Schedule


def test_default_schedule_stages():
    s = Schedule()
    stages = [it for it in range(1, 16001) if s.stage_at(it)]
    assert stages[0] == 500 and stages[1] == 600 and stages[-1] == 15000
    assert len(stages) == (15000 - 500) // 100 + 1
    assert all(b - a == 100 for a, b in zip(stages, stages[1:]))
    assert not any(s.stage_at(it) for it in range(1, 500))


def test_short_schedule_stages():
    s = Schedule(warmup=3, interval=2, densify_until=9)
    assert [it for it in range(1, 20) if s.stage_at(it)] == [3, 5, 7, 9]


def test_densify_limits_in_log_domain():
    p = DensifyLimits().params(extent=4.0)
    assert math.isclose(p.log_dense_scale, math.log(0.04))
    assert math.isclose(p.opacity_logit_min, math.log(0.005 / 0.995))
    assert p.log_max_scale == float("inf") and p.split_n == 2
    assert math.isclose(p.log_shrink, math.log(1.6))
    assert abs(p.grad_threshold - 2e-4) < 1e-9
    q = DensifyLimits(max_fraction=0.1).params(extent=4.0)
    assert math.isclose(q.log_max_scale, math.log(0.4))
