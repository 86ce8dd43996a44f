"""Host logic of bench.py: the committed HBM traffic record applies only to the
scoring kernel's code it was measured on, and only to its workload."""
import bench


def test_code_only_ignores_comments_and_blank_lines():
    a = "int x = 1;  // one\n\n// a comment line\nfloat y = 2.f;\n"
    b = "int x = 1;\n  // reworded comment\nfloat y = 2.f;   \n\n"
    c = "int x = 2;\nfloat y = 2.f;\n"
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only(a) != bench._code_only(c)
    assert bench._code_only(a) == "int x = 1;\nfloat y = 2.f;"


def _recorded_hash():
    import os
    path = os.path.join(bench.ROOT, "profiles", "score_kernel_config1_traffic.txt")
    for line in open(path):
        if line.startswith("kernel_hash"):
            return line.split("=", 1)[1].strip()
    raise AssertionError("no kernel_hash in the traffic record")


def test_recorded_traffic_applies_to_its_workload_only(monkeypatch):
    # as if the kernel code were the one the record was taken on
    monkeypatch.setattr(bench, "kernel_source_hash", _recorded_hash)
    t = bench.recorded_traffic(10_000_000)
    assert t is not None and t > 0
    assert bench.recorded_traffic(9_999_999) is None


def test_recorded_traffic_refuses_a_changed_kernel(monkeypatch):
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0000000000000000")
    assert bench.recorded_traffic(10_000_000) is None


def test_valu_record_applies_to_its_kernel_only(monkeypatch):
    import os
    path = os.path.join(bench.ROOT, "profiles", "score_kernel_config1_valu.txt")
    h = [ln.split("=", 1)[1].strip() for ln in open(path) if ln.startswith("kernel_hash")][0]
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    v = bench.recorded_valu(10_000_000)
    assert v is not None and 0 < v["valu_busy_pair_probe"] and 0 < v["valu_busy"]
    assert bench.recorded_valu(10_000_001) is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0000000000000000")
    assert bench.recorded_valu(10_000_000) is None


def test_bound_follows_the_larger_counter_share():
    v = {"valu_busy": 1.2, "valu_busy_pair_probe": 1.1, "valu_utilization": 1.0, "valu_insts_per_pose": 400.0}
    assert bench.choose_bound(0.8, v) == "alu"     # 1.2 / 1.1 of the probe's busy share
    assert bench.choose_bound(1.1, v) == "hbm"
    assert bench.choose_bound(None, v) is None
    assert bench.choose_bound(0.5, None) is None


def test_roofline_record_names_the_bound_of_the_committed_records(monkeypatch):
    """With the committed counter records of the scoring kernel's code and the
    benchmark workload (1e7 poses of a 40-atom, 604-pair, 10-torsion ligand):
    both resources are near their limits and the VALU's share is the larger, so
    the headline leg is the ALU one; the HBM leg and the traffic sit beside it."""
    import os
    path = os.path.join(bench.ROOT, "profiles", "score_kernel_config1_valu.txt")
    h = [ln.split("=", 1)[1].strip() for ln in open(path) if ln.startswith("kernel_hash")][0]
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    r = bench.roofline_record(6.88, 10_000_000, 40, 604, 10)
    assert r["bound"] == "alu" and r["unit"] == "T VALU lane-instr/s"
    assert r["frac"] == r["alu"]["frac"] and 0.5 < r["frac"] < 1.0
    assert r["achieved"] == round(20720 * 1e7 / 6.88e-3 / 1e12, 2)
    assert 0.8 < r["traffic_frac"] < 1.0 and r["traffic"] > 3.84e10
    assert r["hbm"]["unit"] == "GB/s" and r["alu"]["executed"]["frac"] > r["alu"]["frac"]
    # other kernel code: no records, the HBM leg by default, said so
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0000000000000000")
    r = bench.roofline_record(6.88, 10_000_000, 40, 604, 10)
    assert r["bound"] == "hbm" and r["traffic"] is None and r["bound_source"].startswith("none")
