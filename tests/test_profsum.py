"""Host logic of the rocprofv3 summariser (profiles/ are written by it):
name demangling, bandwidth and clock arithmetic on synthetic CSV rows."""
import csv

import pytest

from paper_2006_14080_amd import profsum


def _write(path, header, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(header)
        w.writerows(rows)
    return str(path)


def test_split_kernel_names_are_unmangled():
    bf = "_ZN3mri12_GLOBAL__N_110nudft_adj8INS0_8PolSplitIDF16bLb0EEELi4EEEvNS_10NudftTableE"
    f16 = "_ZN3mri12_GLOBAL__N_19nudft_fwdINS0_8PolSplitIDF16_Lb1EEELi4EEEvNS_10NudftTableE"
    assert profsum.short(bf) == "nudft_adj8<PolBF16, 4>(mri::NudftTable)"
    assert profsum.short(f16) == "nudft_fwd<PolF16, 4>(mri::NudftTable)"
    assert profsum.short("void mri::(anonymous namespace)::k_cg_dir(mri::SolveTable)") == "k_cg_dir(mri::SolveTable)"


def test_run_sizes_takes_the_last_size_line(tmp_path):
    log = tmp_path / "run.log"
    log.write_text("npix=10 coils=2 planes=3\nnoise\nprofile driver done: npix=94371840 coils=1 planes=1\n")
    assert profsum.run_sizes(str(log)) == (94371840, 1, 1)
    (tmp_path / "empty.log").write_text("nothing\n")
    with pytest.raises(SystemExit):
        profsum.run_sizes(str(tmp_path / "empty.log"))


def test_vecbw_rate_from_algorithmic_bytes(tmp_path):
    # k_cg_update moves 48 B per pixel; 1e8 pixels in 1 ms is 4.8 TB/s = 60 % of 8 TB/s.
    hdr = ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs"]
    p = _write(tmp_path / "s.csv", hdr, [["k_cg_update(mri::SolveTable)", 5, 5e6, 1e6, 50.0, 1e6, 1e6]])
    out = profsum.vecbw(p, 100_000_000, 1, 1)
    line = [x for x in out if x.startswith("k_cg_update")][0]
    assert "4800.0" in line and "60.0%" in line
    # A rate above the HBM peak means the byte count is wrong: refused.
    p = _write(tmp_path / "t.csv", hdr, [["k_cg_update(mri::SolveTable)", 5, 5e5, 1e5, 50.0, 1e5, 1e5]])
    with pytest.raises(SystemExit):
        profsum.vecbw(p, 100_000_000, 1, 1)


def test_clock_and_busy_fraction(tmp_path):
    # Dispatches at 2.0 GHz per die (GRBM summed over the dies) with the matrix
    # cores busy 60 % of the SIMD cycles: 0.5 of the cycles at 2.4 GHz.
    name = "_ZN3mri12_GLOBAL__N_19nudft_fwdINS0_8PolSplitIDF16bLb0EEELi4EEEvNS_10NudftTableE"
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    rows = []
    for i in range(8):
        us = 300.0 + i
        cycles = 2.0e3 * us
        rows += [[i, name, "GRBM_GUI_ACTIVE", profsum.XCDS * cycles, 1000, 1000 + int(us * 1000)],
                 [i, name, "SQ_VALU_MFMA_BUSY_CYCLES", 0.6 * profsum.SIMDS * cycles, 1000, 1000 + int(us * 1000)]]
    rows.append([99, "k_cg_dir(mri::SolveTable)", "GRBM_GUI_ACTIVE", 1.0, 0, 1000])
    out = profsum.clock(_write(tmp_path / "c.csv", hdr, rows))
    assert out[0] == "nudft_fwd<PolBF16, 4>(mri::NudftTable): 8 dispatches"
    quart = [x.split() for x in out if x.strip().startswith("Q")]
    assert len(quart) == 4
    for q in quart:
        assert float(q[2]) == pytest.approx(2.0, abs=1e-3)
        assert float(q[3]) == pytest.approx(0.5, abs=1e-3)
        assert float(q[4]) == pytest.approx(0.6, abs=1e-3)


def test_busy_window_is_the_union_of_kernel_intervals(tmp_path):
    hdr = ["Kernel_Name", "Start_Timestamp", "End_Timestamp"]
    rows = [["nudft_fwd", 0, 100], ["k_mu", 50, 150], ["k_rhs", 300, 400], ["nudft_adj8", 900, 1000]]
    out = profsum.busy(_write(tmp_path / "k.csv", hdr, rows), 10)
    assert out[0].startswith("window 0.00 s") and "(35.0%)" in out[0]


def test_fingerprint_ignores_comments_and_whitespace():
    assert profsum._code_only("int a; // note\n  int  b;\n") == "inta;intb;"
