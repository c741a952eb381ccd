"""The rocprofv3 summary tool on a small synthetic kernel trace (CPU)."""
import csv
import io
import contextlib

from paper_1801_08655_amd import rocprof_summary as rs


def _trace(tmp_path, rows):
    d = tmp_path / "kt"
    d.mkdir()
    with open(d / "kt_kernel_trace.csv", "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp", "Stream_Id"])
        for i, (name, s, e) in enumerate(rows):
            w.writerow([i + 1, name, s, e, 0])
    return str(d)


def _run(argv):
    out = io.StringIO()
    with contextlib.redirect_stdout(out):
        rs.main(argv)
    return out.getvalue()


def test_short_names():
    assert rs._short("void helm::kern::(anonymous namespace)::k_fwd_gemm<float, 64, true>"
                     "(helm::FrontDev const*, int)") == "k_fwd_gemm<float, 64, true>"
    assert rs._short("helm::kern::(anonymous namespace)::k_add(HIP_vector_type<double, 2u>*)") == "k_add"
    assert rs._short("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"


def test_timeline_window_and_top(tmp_path):
    # two steps of [gemm 0-100, other 100-130, gap, ...]; the window from the
    # 2nd last gemm to the last one holds the first step only
    rows = [("void k_fwd_gemm<float>(int)", 0, 100), ("k_jump(int)", 100, 130),
            ("void k_fwd_gemm<float>(int)", 200, 300), ("k_jump(int)", 300, 310)]
    d = _trace(tmp_path, rows)
    out = _run(["timeline", d, "--class", "gemm=k_fwd_gemm", "--window-match", "k_fwd_gemm",
                "--window-from", "2", "--window-to", "1", "--top", "2"])
    assert "dispatches: 2;" in out
    assert "span 0.000 s" in out
    assert "| gemm | 1 | 0.0 | 0.0 | 1.00 | - |" in out
    lines = [l for l in out.splitlines() if l.startswith("| `")]
    assert lines[0].startswith("| `k_fwd_gemm<float>` | 1 |") and lines[0].endswith("| 0.769 |")
    assert lines[1].startswith("| `k_jump` | 1 |") and lines[1].endswith("| 0.231 |")
