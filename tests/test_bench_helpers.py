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


def test_traffic_is_keyed_by_source_workload_and_shape(monkeypatch):
    """A figure is reported only for the integrator source its counters were
    taken on, and only for its own workload and launch shape."""
    table = bench.TRAFFIC["bytes_per_launch"]
    monkeypatch.setattr(bench, "TRAFFIC", {"source_sha256": "a" * 64,
                                           "bytes_per_launch": {"orbit": {(256, 8): 123}}})
    monkeypatch.setattr(bench, "integrator_source_hash", lambda: "a" * 64)
    assert bench.traffic_for("orbit", (256, 8)) == 123
    assert bench.traffic_for("orbit", [256, 8]) == 123
    assert bench.traffic_for("orbit", (128, 8)) is None
    assert bench.traffic_for("orbit") is None
    assert bench.traffic_for("batched", (256, 8)) is None
    monkeypatch.setattr(bench, "integrator_source_hash", lambda: "b" * 64)
    assert bench.traffic_for("orbit", (256, 8)) is None
    # the committed figures, if any, are per-launch byte counts of plausible size
    for per_shape in table.values():
        for shape, nbytes in per_shape.items():
            assert len(shape) == 2 and 1e6 < nbytes < 1e11


def test_flop_counts():
    # DP45: 6 derivative evaluations plus the fixed combination; RK4: 4
    for kind in range(4):
        assert bench.attempt_flops(kind, 1) == bench.DP45_COMBINE_FLOPS + 6 * bench.ACCEL_FLOPS[kind]
        assert bench.attempt_flops(kind, 0) == bench.RK4_COMBINE_FLOPS + 4 * bench.ACCEL_FLOPS[kind]
    assert bench.ACCEL_FLOPS[0] == 0  # radial-o: straight chords
    # the reduced radial terms: azimuthal-e cheapest of the curved branches
    assert bench.ACCEL_FLOPS[3] < bench.ACCEL_FLOPS[1] < bench.ACCEL_FLOPS[2]
    assert math.isclose(bench.PEAK_FP64_TFLOPS, 256 * 2.4e9 * 128 / 1e12, rel_tol=1e-3)
