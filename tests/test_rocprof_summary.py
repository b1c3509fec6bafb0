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


def test_valu_only_for_the_profiled_source(tmp_path):
    sha = "ab" * 32
    p = tmp_path / "v.md"
    p.write_text(f"x\nsource_sha256: {sha}\n\n```\nvalu_insts k_push<double>: 66529503\n"
                 f"valu_busy k_push<double>: 45.18\nvalu_insts k_push_fixed: 73264383\n```\n")
    assert R.read_valu(str(p), "k_push<double>", sha) == (66529503, 45.18)
    assert R.read_valu(str(p), "k_push_fixed", sha) == (73264383, None)
    assert R.read_valu(str(p), "k_push<float>", sha) is None
    assert R.read_valu(str(p), "k_push<double>", "cd" * 32) is None
    assert R.read_valu(str(tmp_path / "missing.md"), "k_push<double>", sha) is None


def test_valu_summary_from_counter_csv(tmp_path):
    """A counter CSV as rocprofv3 writes it (one row per dispatch and counter)
    condenses to per-kernel means and the machine-readable lines bench reads."""
    d = tmp_path / "run"
    d.mkdir()
    hdr = ('"Correlation_Id","Dispatch_Id","Agent_Id","Queue_Id","Process_Id","Thread_Id","Grid_Size",'
           '"Kernel_Id","Kernel_Name","Workgroup_Size","LDS_Block_Size","Scratch_Size","VGPR_Count",'
           '"Accum_VGPR_Count","SGPR_Count","Counter_Name","Counter_Value","Start_Timestamp","End_Timestamp"')
    rows = [hdr]
    k = '"void (anonymous namespace)::k_push<double>((anonymous namespace)::StepArgs<double>, int)"'
    for disp, (waves, insts, busy) in enumerate([(100, 40000, 40.0), (100, 44000, 50.0)]):
        for c, v in (("SQ_WAVES", waves), ("SQ_INSTS_VALU", insts), ("VALUBusy", busy)):
            rows.append(f'{disp},{disp},"Agent 1",1,1,1,6400,7,{k},256,0,0,66,0,64,"{c}",{v},0,1')
    (d / "bench_counter_collection.csv").write_text("\n".join(rows) + "\n")
    sha = "ef" * 32
    text = R.valu_summary(str(d), "bench", "cmd", sha)
    out = tmp_path / "s.md"
    out.write_text(text)
    assert "| `k_push<double>` | 2 | 100 | 4.2e+04 | 420.0 | 45.0 |" in text
    assert R.read_valu(str(out), "k_push<double>", sha) == (42000, 45.0)


def test_committed_counter_summaries_match_the_source():
    """Every committed counter summary that bench.py reads was taken on the
    HIP source as it stands and names the particle kernels bench reports for
    its workload (so the roofline's traffic and VALU figures are not null)."""
    import bench
    sha = R.source_sha256()
    expect = {"40cube": ["k_push<double>", "k_push<float>", "k_push_fixed"],
              "precision": ["k_push<double>", "k_push<float>", "k_push_fixed"],
              "large-box": ["k_push<double>", "k_push_pipe<false>", "k_push_pipe<true>"]}
    for key, (traffic, valu) in bench.PROFILE_SUMMARIES.items():
        for k in expect[key]:
            assert R.read_traffic(traffic, k, sha) is not None, (key, k, traffic)
            assert R.read_valu(valu, k, sha) is not None, (key, k, valu)
