"""Host-side logic of the benchmark, without a GPU: the one-GPU guard, the
HBM-traffic figure's validity check, the comparison counts it reports, and
the CPU baseline's fields on a tiny sample."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import workload as wl  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr and r.stdout == ""


def test_dot_traffic_only_for_the_measured_kernel_and_workload():
    t = bench.dot_traffic(1984, 300_000, 0)
    assert t is not None
    # the stored passes: FETCH_SIZE scaled x2 (copy calibration), WRITE_SIZE x1
    assert 36.5e9 < t < 37.5e9
    # never below the algorithmic bytes: the 30.72 GB region is read at least
    # once per launch (far larger than the caches) and the outputs written once
    assert t >= 300_000 * 102_400 + 2 * 2 * 1984 * 300_000
    assert bench.dot_traffic(1984, 300_001, 0) is None
    assert bench.dot_traffic(992, 300_000, 0) is None
    assert bench.dot_traffic(1984, 300_000, 1) is None       # an expanded tile configuration


def test_reported_op_counts():
    # 2 vectors x 25,600 k x 3 limb products x 2 ops per comparison and party
    assert bench.OPS_PER_CMP_PARTY == 307_200
    assert bench.DB_BYTES_PER_ENTRY_PARTY == 102_400
    # ChaCha12: 12 rounds x 4 quarter-rounds x 12 int ops + 16 final adds
    assert bench.CHACHA12_OPS == 592
    assert abs(bench.VALU_PEAK_TOPS - 39.3216) < 1e-9


def test_cpu_baseline_fields_on_a_tiny_sample():
    w = wl.full_protocol(n_db=1024, n_q=2)
    qc, qm = wl.make_queries(w)
    r = bench.cpu_baseline(w, qc, qm, sample_q=1, sample_n=64)
    assert r["kind"] == "oracle" and r["unit"] == "comparisons/s" and r["cores"] >= 1
    assert r["value"] > 0 and "1 queries x 31 rotations x 64 entries" in r["sample"]
    assert r["single_core"]["value"] > 0 and r["plaintext_check"]["single_core"] > 0
    assert isinstance(r["cpu_model"], str)
    import oracle as orc

    assert orc.threads() == r["cores"]          # the single-thread timing restored the thread count


def test_in_batch_planting_targets_earlier_queries():
    import oracle as orc

    w = wl.full_protocol(n_db=1024, n_q=16)
    qc, qm = wl.make_queries(w)
    wl.plant_in_batch(w, qc, qm)
    dups = [int(orc.plain(qc[i:i + 1], qm[i:i + 1], w.rot, qc[:i], qm[:i])[3][0]) for i in (9, 11, 13, 15)]
    assert dups == [1, 1, 0, 0]                # HD 0.20 and 0.30 match; 0.42 and the exact threshold do not
    assert np.array_equal(wl.make_queries(w)[0][:9], qc[:9])


def test_two_eye_recipe_plants_every_pattern():
    """The two-eye workload: 32 persons of two queries, database plants by
    the left eye, the right eye and both, and in-batch pairs whose plaintext
    decisions (each eye against the eyes of earlier persons) are the ones the
    recipe names: 22, 39 and 55 count, 31 (a right eye made from its own left
    eye) and 46 (made from a later person's eye) and 62 (exactly at the
    threshold) do not."""
    import oracle as orc

    w = wl.two_eyes(n_db=1024)
    assert (w.n_q, w.group, len(w.rot)) == (64, 2, 31)
    by_person = {}
    for qi, _, _, hx in w.planted:
        by_person.setdefault(qi // 2, set()).add(qi % 2)
    assert by_person[0] >= {0} and by_person[1] >= {1} and by_person[2] == {0, 1}
    assert 15 not in by_person and 23 not in by_person and 27 not in by_person
    assert {(3, "eq"), (7, "lt")} <= {(qi // 2, hx) for qi, _, _, hx in w.planted if isinstance(hx, str)}
    qc, qm = wl.make_queries(w)
    wl.plant_in_batch(w, qc, qm, w.batch_pairs)
    got = {}
    for i in (22, 31, 39, 46, 55, 62):
        k = 2 * (i // 2)
        got[i] = int(orc.plain(qc[i:i + 1], qm[i:i + 1], w.rot, qc[:k], qm[:k])[3][0])
    assert got == {22: 1, 31: 0, 39: 1, 46: 0, 55: 1, 62: 0}
    # with groups of one, the right eye made from its own left eye would count
    assert int(orc.plain(qc[31:32], qm[31:32], w.rot, qc[:31], qm[:31])[3][0]) == 1


def test_served_latency_probe_runs_with_the_default_workload_only():
    """The probe follows the default full workload (MPCLift, one decision per
    query); the other settings and workloads report their own figures."""
    from types import SimpleNamespace

    base = dict(workload="full", compare="mpclift", in_batch=False, two_eyes=False, no_serve_probe=False)
    assert bench.serve_probe_applies(SimpleNamespace(**base))
    for change in (dict(workload="serve"), dict(compare="plain"), dict(in_batch=True), dict(two_eyes=True),
                   dict(no_serve_probe=True)):
        assert not bench.serve_probe_applies(SimpleNamespace(**{**base, **change})), change
    assert bench.SERVE_PROBE_REQUESTS / bench.SERVE_PROBE_RATE == 2.0
