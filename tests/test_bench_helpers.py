"""CPU checks of bench.py's bookkeeping: the JSON it prints is strict, the
HBM traffic it reports belongs to the integrator source and launch shape it
was measured on, and the algorithmic flop counts are consistent."""
import json
import math

import bench


def test_finite_json_is_strict():
    rec = {"a": float("nan"), "b": [1.0, float("inf"), {"c": -float("inf")}], "d": (2.0, 3)}
    out = bench.finite_json(rec)
    assert out == {"a": None, "b": [1.0, None, {"c": None}], "d": [2.0, 3]}
    json.loads(json.dumps(out, allow_nan=False))


def test_traffic_is_keyed_by_source_and_shape(monkeypatch):
    shapes = bench.TRAFFIC["bytes_per_launch"]
    if bench.TRAFFIC["source_sha256"] != bench.integrator_source_hash():
        # counters taken on another integrator source: no figure is reported
        assert bench.traffic_for(256, 2) == (None, None)
        monkeypatch.setattr(bench, "integrator_source_hash", lambda: bench.TRAFFIC["source_sha256"])
    # every measured shape reports its own figure
    for (block, refill), nbytes in shapes.items():
        assert bench.traffic_for(block, refill) == (nbytes, [block, refill])
    # another shape reports the nearest measured one, and names it
    t, shape = bench.traffic_for(64, 1)
    assert tuple(shape) in shapes and t == shapes[tuple(shape)]
    # a changed integrator source reports no traffic
    monkeypatch.setattr(bench, "integrator_source_hash", lambda: "0" * 64)
    assert bench.traffic_for(256, 2) == (None, None)


def test_traffic_figures_are_plausible():
    """Slot state read and written per entering ray is ~156 B (x, v, t, h,
    counters); the measured 767-790 MB per launch of 3.69 M entering rays is
    208-214 B per ray."""
    for nbytes in bench.TRAFFIC["bytes_per_launch"].values():
        assert 150 < nbytes / 3_688_996 < 260


def test_flop_counts():
    # DP45: 6 derivative evaluations plus the fixed combination; RK4: 4
    for kind in range(4):
        assert bench.attempt_flops(kind, 1) == bench.DP45_COMBINE_FLOPS + 6 * bench.ACCEL_FLOPS[kind]
        assert bench.attempt_flops(kind, 0) == bench.RK4_COMBINE_FLOPS + 4 * bench.ACCEL_FLOPS[kind]
    assert bench.ACCEL_FLOPS[0] == 0  # radial-o: straight chords
    # the reduced radial terms: azimuthal-e cheapest of the curved branches
    assert bench.ACCEL_FLOPS[3] < bench.ACCEL_FLOPS[1] < bench.ACCEL_FLOPS[2]
    assert math.isclose(bench.PEAK_FP64_TFLOPS, 256 * 2.4e9 * 128 / 1e12, rel_tol=1e-3)
