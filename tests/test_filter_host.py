"""The complete-graph scan's float filter and box culling test
(paper_2011_08170_amd/csrc/f2m_filter.h), compiled for the host: on
adversarial inputs -- full 2^20 coordinate span, |Lam| up to 2^37,
thresholds at, just above and just below each pair's exact Z, distances at
the EUC_2D rounding boundaries -- no pair with Z <= theta + slack is ever
skipped (the method needs every such pair exactly)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2011_08170_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_filter_and_culling_are_conservative(tmp_path):
    exe = str(tmp_path / "filter_check")
    subprocess.run([HIPCC, "-O2", "-std=c++17", "-I", CSRC, os.path.join(HERE, "native", "filter_check.cpp"),
                    "-o", exe], check=True, capture_output=True)
    out = subprocess.run([exe, "400000"], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        parts = line.split()
        if len(parts) == 4 and parts[0] in ("filter", "box"):
            got[parts[0]] = [int(x) for x in parts[1:]]
    for name in ("filter", "box"):
        checked, tight, bad = got[name]
        assert checked > 3_000_000 and tight > 500_000, (name, got)
        assert bad == 0, out
