"""Host-side checks of the benchmark driver (no GPU): the step schedule never takes the circuit
beyond its depth, and the multi-GPU request is refused with a message."""

import bench


def test_schedule_replays_saturated_layers_from_the_checkpoint():
    sched = bench.step_schedule(9, 20, 25)
    assert [li for li, _ in sched[:11]] == list(range(9, 20))
    assert all(9 <= li < 20 for li, _ in sched)          # depth never exceeds 20
    assert [j for j, (_, imp) in enumerate(sched) if imp] == [11, 22]
    assert sched[11][0] == 9 and sched[22][0] == 9        # a pass restarts at layer 10


def test_setup_layers_reach_saturation():
    assert bench.setup_layers(256) == 9
    assert bench.setup_layers(64) == 7


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU" in capsys.readouterr().err


def test_reference_counts():
    assert bench.svd_reference_flops(256) == 88.0 * 512 ** 3
    assert bench.theta_flops(256) == 32.0 * 256 ** 3 + 128.0 * 256 ** 2
