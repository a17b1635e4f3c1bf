"""Host logic of the staggered KNN radius schedule (Section 3.5.2): the radius pfn_train_field
uses at each step, checked against the proportions of the paper's Table 1 (four stages over
0-36 %, 37-63 %, 64-90 % and 91-100 % of the steps, radii growing to the final one in the
ratios 1 : 2 : 4 : 8 of its 12M-photon row).  No GPU is needed."""
import pytest

from paper_2304_07338_amd.pfn import PfnError, TrainConfig, train_step_radius


def test_staggered_stages():
    cfg = TrainConfig(steps=1000, target="photon_map", radius=0.08, staggered=True, knn_k=1024)
    expect = {0: 0.01, 359: 0.01, 360: 0.02, 629: 0.02, 630: 0.04, 899: 0.04, 900: 0.08,
              999: 0.08}
    for step, r in expect.items():
        assert train_step_radius(cfg, step) == pytest.approx(r, rel=1e-6), step
    # the stage ratios of Table 1's 12M row: 0.25, 0.5, 1.0, 2.0
    rs = [train_step_radius(cfg, s) for s in (0, 400, 700, 950)]
    assert [r / rs[-1] for r in rs] == pytest.approx([0.125, 0.25, 0.5, 1.0])


def test_naive_schedule_keeps_the_final_radius():
    cfg = TrainConfig(steps=30, target="photon_map", radius=0.05, staggered=False)
    for s in range(30):
        assert train_step_radius(cfg, s) == pytest.approx(0.05, rel=1e-6)


def test_out_of_range_step_is_rejected():
    cfg = TrainConfig(steps=10, target="photon_map", radius=0.05, staggered=True)
    with pytest.raises(PfnError):
        train_step_radius(cfg, 10)
    with pytest.raises(PfnError):
        train_step_radius(cfg, -1)


@pytest.mark.parametrize("step", [0, 1, 1399, 1400, 1424, 1425, 1426, 1449, 1450, 1999])
def test_learning_rate_schedule_matches_oracle(orc, step):
    """The rate pfn_train_field hands to Adam at `step` (Section 3.5.1: 9e-4, x0.92 from 70 % of
    2000 steps and every 25 steps after) equals the oracle's schedule, rounded once to FP32."""
    import numpy as np
    from paper_2304_07338_amd.pfn import train_lr_at
    cfg = TrainConfig()
    got = train_lr_at(cfg, step)
    # the parameter block carries lr and decay as FP32
    ref = orc.lr_at(step, np.float32(cfg.lr), np.float32(cfg.decay), cfg.decay_start,
                    cfg.decay_interval)
    assert got == np.float32(ref), (step, got, ref)
    closed = {0: 9e-4, 1399: 9e-4, 1400: 9e-4 * 0.92, 1424: 9e-4 * 0.92, 1425: 9e-4 * 0.92 ** 2,
              1999: 9e-4 * 0.92 ** 24}
    if step in closed:
        assert got == pytest.approx(closed[step], rel=1e-6)


def test_learning_rate_schedule_other_settings(orc):
    import numpy as np
    from paper_2304_07338_amd.pfn import train_lr_at
    cfg = TrainConfig(steps=300, lr=1e-2, decay=0.5, decay_start=100, decay_interval=7)
    for step in range(300):
        ref = orc.lr_at(step, np.float32(cfg.lr), np.float32(cfg.decay), cfg.decay_start,
                        cfg.decay_interval)
        assert train_lr_at(cfg, step) == np.float32(ref), step


def test_learning_rate_bad_arguments_are_rejected():
    from paper_2304_07338_amd.pfn import train_lr_at
    with pytest.raises(PfnError):
        train_lr_at(TrainConfig(steps=10), 10)
    with pytest.raises(PfnError):
        train_lr_at(TrainConfig(steps=10, decay_interval=0), 3)
