"""Host-side parts of the measurement: bench.py's one-GPU contract and the
rocprofv3 summary parsers that feed its roofline fields (CPU only)."""
import os
import subprocess
import sys

from paper_1208_2428_amd import profsum

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""  # no JSON line for a configuration it cannot run


def test_trace_and_counter_summaries(tmp_path):
    stats = tmp_path / "run_kernel_stats.csv"
    stats.write_text('"Name","Calls","TotalDurationNs","AverageNs","Percentage"\n'
                     '"void fhp::(anonymous namespace)::k_stepk<5, true, true, 0, false>'
                     '(unsigned long const*, unsigned long*, unsigned long const*, '
                     'fhp::StepkArgs)",4,520000,130000.0,99.0\n')
    assert profsum.trace_summary(str(stats)) == [("k_stepk<5, true, true, 0, false>", 4, 130.0)]
    pmc = tmp_path / "run_counter_collection.csv"
    pmc.write_text('"Kernel_Name","Counter_Name","Counter_Value"\n'
                   '"k_stepk<5, true, true, 0, false>(args)","FETCH_SIZE",100.0\n'
                   '"k_stepk<5, true, true, 0, false>(args)","FETCH_SIZE",300.0\n'
                   '"k_init(args)","FETCH_SIZE",7.0\n')
    assert profsum.pmc_summary(str(pmc), "k_stepk") == {
        ("k_stepk<5, true, true, 0, false>", "FETCH_SIZE"): (2, 200.0)}


def test_recorded_profile_fields():
    """The committed note of the headline kernel carries the figures bench.py
    reads: HBM bytes per launch, VALU instructions per launch, the depth and
    the source hash they were taken on."""
    md = os.path.join(ROOT, "profiles", "k_stepk_porous-16384.md")
    traffic, src, depth = profsum.recorded_traffic(md)
    assert traffic and traffic > 4.7e8  # at least the algorithmic bytes of a 16384^2 pass
    assert depth == 5 and src and len(src) == 12
    assert profsum.recorded_value(md, "valu_insts_per_launch") > 0


def test_build_flags_and_kernel_sources_name_existing_files():
    """Per-source compiler flags and the sources whose hash gates the recorded
    traffic must name files that exist (a renamed source would otherwise drop
    its flags, or leave the recorded traffic gated on nothing)."""
    import os
    from paper_1208_2428_amd import build
    names = {os.path.basename(p) for p in build.sources()}
    assert set(build.FILE_FLAGS) <= names
    for rel in profsum.KERNEL_SOURCES:
        assert os.path.exists(os.path.join(profsum.PKG, rel)), rel
    assert "csrc/fhp_stepk_k5.hip" in profsum.KERNEL_SOURCES
