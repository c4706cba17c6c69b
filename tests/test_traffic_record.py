"""Host-side checks of the HBM-traffic records (paper_1710_07041_amd.traffic):
the copy calibration scales each counter to bytes, dispatches of one kernel
class average, unknown kernels are ignored, and the source digest ignores
comments but not code."""
import csv
import json

import pytest

from paper_1710_07041_amd import traffic


def write_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, kib in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": kib})


def test_scaling_and_averaging(tmp_path):
    gib_kib = (1 << 30) / 1024.0
    # the calibration copy reads half of its bytes per FETCH_SIZE unit and
    # writes exactly its bytes; two sweep dispatches average
    fetch = [("void at::native::copyBuffer(float*)", gib_kib / 2),
             ("void dd::(anonymous namespace)::k_sap_sweep<__half, float, X>(...)", 1000.0),
             ("void dd::(anonymous namespace)::k_sap_sweep<__half, float, X>(...)", 3000.0),
             ("void dd::(anonymous namespace)::k_unrelated(...)", 5.0)]
    write = [("void at::native::copyBuffer(float*)", gib_kib),
             ("void dd::(anonymous namespace)::k_sap_sweep<__half, float, X>(...)", 500.0),
             ("void dd::(anonymous namespace)::k_sap_sweep<__half, float, X>(...)", 500.0)]
    fp, wp, out = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "t.json"
    write_csv(fp, "FETCH_SIZE", fetch)
    write_csv(wp, "WRITE_SIZE", write)
    traffic.main(str(fp), str(wp), str(out), "cmd")
    rec = json.loads(out.read_text())
    assert rec["copy_calibration"]["fetch_scale"] == pytest.approx(2.0)
    assert rec["copy_calibration"]["write_scale"] == pytest.approx(1.0)
    k = rec["kernels"]
    assert set(k) == {"sap_sweep_f16"}
    assert k["sap_sweep_f16"]["dispatches"] == 2
    assert k["sap_sweep_f16"]["traffic_bytes"] == pytest.approx(2000.0 * 1024 * 2 + 500.0 * 1024, rel=1e-9)
    assert rec["source_digest"] == traffic.source_digest()


def test_missing_calibration_copy_is_an_error(tmp_path):
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    write_csv(fp, "FETCH_SIZE", [("void dd::k_dslash<double, double, X>(...)", 1.0)])
    write_csv(wp, "WRITE_SIZE", [("void dd::k_dslash<double, double, X>(...)", 1.0)])
    with pytest.raises(SystemExit):
        traffic.main(str(fp), str(wp), str(tmp_path / "t.json"), "cmd")


def test_digest_ignores_comments_only():
    code = "int f(int a)\n{\n    return a + 1;\n}\n"
    commented = "// a comment\nint f(int a) /* inline */\n{\n\n    return a + 1; // trailing\n}\n"
    changed = "int f(int a)\n{\n    return a + 2;\n}\n"
    assert traffic._code_only(code) == traffic._code_only(commented)
    assert traffic._code_only(code) != traffic._code_only(changed)


def test_kernel_classes():
    assert traffic.classify("void dd::(anonymous namespace)::k_dslash<float, double, double, double, false>(x)") \
        == "dslash_f32in_f64"
    assert traffic.classify("void dd::(anonymous namespace)::k_dslash<double, double, double, double>(x)") == "dslash_f64"
    assert traffic.classify("void dd::(anonymous namespace)::k_sap_sweep<float, float, R, float>(x)") == "sap_sweep_f32"
    assert traffic.classify("void dd::(anonymous namespace)::k_dots_lag<3>(x)") == "cgs_dots"
    assert traffic.classify("void something_else()") is None
