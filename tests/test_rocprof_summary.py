"""The counter summary parser that bench.py uses for the roofline's traffic field."""
import os

from paper_2208_12795_amd import rocprof_summary as R

PROFILE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles",
                       "k_push_hbm_traffic_40cube_1e7.md")


def test_traffic_only_for_the_profiled_source(tmp_path):
    sha = "ab" * 32
    p = tmp_path / "t.md"
    p.write_text(f"x\nsource_sha256: {sha}\n\n```\ntraffic_bytes k_push<double>: 1234\n"
                 f"traffic_bytes k_push<float>: 99\n```\n")
    assert R.read_traffic(str(p), "k_push<double>", sha) == 1234
    assert R.read_traffic(str(p), "k_push<float>", sha) == 99
    assert R.read_traffic(str(p), "k_walk<float>", sha) is None
    assert R.read_traffic(str(p), "k_push<double>", "cd" * 32) is None
    assert R.read_traffic(str(tmp_path / "missing.md"), "k_push<double>", sha) is None


def test_committed_profile_parses():
    text = open(PROFILE).read()
    assert "source_sha256:" in text and "traffic_bytes k_push<double>:" in text
    assert "__amd_rocclr_copyBuffer" in text
