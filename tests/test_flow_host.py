"""Host-side driver logic of paper_2208_08903_amd.flow (no GPU)."""


def test_lr_schedules_closed_form():
    from paper_2208_08903_amd import flow as fl
    s = fl.step_lr(0.5, 2)
    assert [s(1e-3, t) for t in range(1, 7)] == [1e-3, 1e-3, 5e-4, 5e-4, 2.5e-4, 2.5e-4]
    e = fl.exp_lr(0.9)
    assert e(2.0, 1) == 2.0 and abs(e(2.0, 3) - 2.0 * 0.81) < 1e-15
