"""Host-side checks of the rocprofv3 summary tool (synthetic CSV files)."""
import csv
import json

from paper_2608_29082_amd import pmc_summary as P

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _counters(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for i, (k, c, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


def test_short_name_strips_return_type_and_parameters():
    assert P.short_name("void mgl::k_conv_tile<true, false, float, float>(mgl::TileDev, int)") == \
        "mgl::k_conv_tile<true, false, float, float>"
    assert P.short_name("mgl::k_norm_final") == "mgl::k_norm_final"
    assert P.short_name("void f<(anonymous namespace)::T>(int)") == "f<(anonymous namespace)::T>"


def test_traffic_calibration_and_json(tmp_path):
    # the copy reads and writes 256 MiB per dispatch; its FETCH_SIZE reads half of that
    cf, cw = tmp_path / "cf.csv", tmp_path / "cw.csv"
    _counters(cf, [("copyBuffer(x)", "FETCH_SIZE", 131072.0)] * 5)
    _counters(cw, [("copyBuffer(x)", "WRITE_SIZE", 262144.0)] * 5)
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    _counters(f, [("void k<1>(int)", "FETCH_SIZE", 1000.0), ("void k<1>(int)", "FETCH_SIZE", 3000.0),
                  ("void j(int)", "FETCH_SIZE", 10.0)])
    _counters(w, [("void k<1>(int)", "WRITE_SIZE", 500.0), ("void k<1>(int)", "WRITE_SIZE", 500.0)])
    table, cal, per, (ff, fw) = P.traffic(str(f), str(w), str(cf), str(cw), 256)
    assert abs(ff - 2.0) < 1e-12 and abs(fw - 1.0) < 1e-12
    rd, wr = per["k<1>"]
    assert rd == 2000.0 * 2.0 * 1024 and wr == 500.0 * 1024
    assert per["j"] == (10.0 * 2.0 * 1024, 0.0)
    out = tmp_path / "t.json"
    P.main(["traffic", str(f), str(w), str(cf), str(cw), "--kernel", "k<1>", "--json", str(out)])
    rec = json.loads(out.read_text())
    assert rec["bytes_per_dispatch"] == rd + wr
    assert rec["kernel_sources_sha256"] == P.kernel_sources_sha256()


def test_traffic_json_matches_the_kernel_sources():
    # the committed traffic record carries the hash of the sources it was measured on
    import os
    path = os.path.join(os.path.dirname(P.HERE), "profiles", "k_conv_tile_level0_diffusion513_traffic.json")
    rec = json.load(open(path))
    assert rec["kernel"] == "mgl::k_conv_tile<true, false, float, float>"
    assert rec["bytes_per_dispatch"] > 0
