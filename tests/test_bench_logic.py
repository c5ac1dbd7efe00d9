"""Host logic of bench.py (no GPU): the algorithmic byte count and the guard
that reports measured HBM traffic only for the kernel sources it was taken on."""
import bench


def test_vector_passes_of_a_small_schedule_by_hand():
    # p = 2, c = 1, one substep of m = 2.  Stage: b_0..b_2 read, u written (4).
    # Step jj reads x_j, 2 columns of B, 1 field vector and jj basis columns,
    # writes w, then the update reads w and jj + 1 columns and writes x_{jj+1}:
    # 8 for jj = 0, 10 for jj = 1.  Column 0 written once (1).  Combine: 2
    # columns read, 1 written (3).  The result written out (1).
    assert bench.vectors_per_call([(0.1, 2)], 2, 1) == 4 + (8 + 10) + 1 + 3 + 1


def test_vector_passes_of_the_benchmark_call():
    # 14 substeps of m = 64 (the adaptive call at N = 1M): 64545 passes of
    # N float64 = 541.4 GB, the figure the roofline divides by the launch time
    n = 1024 * 1024
    passes = bench.vectors_per_call([(0.1 / 14, 64)] * 14, 2, 1)
    assert passes == 64545
    assert passes * 8 * n == 541442703360


def test_measured_traffic_only_for_matching_sources(tmp_path):
    good = tmp_path / "good.txt"
    good.write_text(f"# comment = ignored\nsource_sha256 = {bench.kernel_source_hash()}\n"
                    "hbm_bytes_per_launch = 1.5e+11\nhbm_bytes_per_call = 2.5e+12\n")
    stale = tmp_path / "stale.txt"
    stale.write_text("source_sha256 = 00\nhbm_bytes_per_launch = 1.5e+11\n")
    assert bench.measured_traffic(str(good)) == 1.5e11
    assert bench.measured_traffic(str(good), "hbm_bytes_per_call") == 2.5e12
    assert bench.measured_traffic(str(stale)) is None
    assert bench.measured_traffic(str(tmp_path / "missing.txt")) is None


def test_committed_summaries_parse():
    """The committed counter summaries carry the source hash they were taken
    on and the byte counts bench.py reads (reported only while the hash
    matches the current sources)."""
    for path, key in ((bench.TRAFFIC_FILE, "hbm_bytes_per_launch"),
                      (bench.BATCH_TRAFFIC_FILE, "hbm_bytes_per_call"),
                      (bench.FP32_TRAFFIC_FILE, "hbm_bytes_per_call")):
        kv = {}
        for line in open(path):
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
        assert len(kv["source_sha256"]) == 64
        assert float(kv[key]) > 0.0


def test_basis_bytes_of_a_small_schedule_by_hand():
    # 4-byte basis, p = 2, c = 1, N = 1, one substep of m = 2.  Stage: 3 float64
    # columns read, u written (32).  Step jj: x_j, jj older columns and w
    # written (basis), 2 columns of B and 1 field (float64), then w, jj + 1
    # columns and x_{jj+1} written (basis): 4 * 5 + 24 = 44 for jj = 0 and
    # 4 * 7 + 24 = 52 for jj = 1.  Column 0 written (4).  Combine: 2 columns
    # read (8), u written (8).  The result written out (8).
    assert bench.basis_bytes_per_call([(0.1, 2)], 2, 1, 1, 4) == 32 + 44 + 52 + 4 + 16 + 8


def test_basis_bytes_with_float64_basis_match_the_vector_passes():
    for sched, p, c in (([(0.1, 2)], 2, 1), ([(0.05, 64)] * 3 + [(0.02, 17)], 2, 2),
                        ([(0.1, 1)], 0, 0), ([(0.01, 48)] * 5, 3, 0)):
        n = 1000
        assert bench.basis_bytes_per_call(sched, p, c, n, 8) == \
            bench.vectors_per_call(sched, p, c) * 8 * n


def test_vector_passes_of_mgs_and_iocgs_by_hand():
    # p = 2, c = 1, one substep of m = 2.  Stage 4, combine 3, out 1 (as above).
    # MGS step 0: matvec reads x_0 (from u), B (2), u (1), writes w and column
    # 0 (2): 6; the norm pass reads w and x_0, writes w: 3 -> 9.  Step 1:
    # matvec reads x_1, B, u, writes w, reads x_0: 6; the second inner product
    # reads w, x_0, x_1 and writes w: 4; the norm pass: 3 -> 13.
    assert bench.vectors_per_call([(0.1, 2)], 2, 1, "mgs") == 4 + (9 + 13) + 3 + 1
    # ioCGS step 0 as MGS (9); step 1: matvec with x_0 . w (6), one pass reads
    # w, x_0, x_1 and writes w (4) -> 10.
    assert bench.vectors_per_call([(0.1, 2)], 2, 1, "iocgs") == 4 + (9 + 10) + 3 + 1
    # the reductions of a step: j + 1 for MGS (Algorithm 1), two for ioCGS
    assert [bench.syncs_per_step(jj, "mgs") for jj in range(3)] == [2, 3, 4]
    assert [bench.syncs_per_step(jj, "iocgs") for jj in range(3)] == [2, 2, 2]
    assert [bench.syncs_per_step(jj, "h-cwy") for jj in range(3)] == [1, 1, 1]


def test_error_metrics():
    import numpy as np
    ref = np.array([1.0, -2.0, 2.0])
    e = bench.errors(ref + np.array([0.0, 0.03, 0.0]), ref)
    assert abs(e["rel_l2"] - 0.01) < 1e-15 and abs(e["max_abs_rel"] - 0.015) < 1e-15


def test_timeline_summary_of_a_synthetic_call():
    """Three phases on three workgroups (stamps in 100 MHz ticks): the start
    phase, then Arnoldi steps j = 1 and 2; every interval checked by hand."""
    import numpy as np
    T = np.zeros((3, 3, 8))
    T[0, 0, [0, 7]] = [100, 200]                  # start phase: released at 200
    T[0, 0, 4] = 0
    for k, (t0, j) in enumerate([(200, 1), (2200, 2)], start=1):
        T[k, 0, 4] = 1000 + j                     # leader: phase code
        T[k, 0, 0] = t0 + 10
        for w, d in ((1, 0), (2, 40)):            # two other workgroups
            T[k, w, 0] = t0 + 100 + d             # release seen
            T[k, w, 1] = t0 + 500 + d             # update done
            T[k, w, 2] = t0 + 600 + d             # flags seen
            T[k, w, 3] = t0 + 1500 + d            # arrival
        T[k, 0, 3] = t0 + 1400
        T[k, 0, 5] = t0 + 1740                    # reduction 200 ticks after the last arrival
        T[k, 0, 6] = t0 + 1900
        T[k, 0, 7] = t0 + 2000                    # release: the next step starts from it
    s = bench.timeline_summary(T)
    assert s["arnoldi_steps"] == 2
    m = s["step_mean_us"]
    assert m["step_us"] == 20.0                   # 2000 ticks = 20 us each
    assert m["release_seen_us"] == 1.2            # median of 100 and 140 ticks
    assert m["update_done_us"] == 5.2 and m["halo_flags_us"] == 6.2
    assert m["arrival_median_us"] == 15.2 and m["arrival_last_us"] == 15.4
    assert m["reduction_after_last_us"] == 2.0
    assert m["serial_us"] == 1.6 and m["release_us"] == 1.0
    assert s["step_fit_us"]["intercept"] == 20.0 and s["step_fit_us"]["per_j"] == 0.0
    assert s["other_phases"] == {}


def test_onchip_bytes_by_hand():
    # 3584 passes kept on chip, N = 1M float64; FP32 basis elements; none
    assert bench.onchip_bytes({"onchip_passes": 3584}, 1 << 20) == 3584 * 8 * (1 << 20)
    assert bench.onchip_bytes({"onchip_passes": 10}, 100, 4) == 10 * 4 * 100
    assert bench.onchip_bytes({"onchip_passes": 0}, 1 << 20) == 0
