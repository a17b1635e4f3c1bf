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
