"""CPU checks of the benchmark's command line (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _summary(path, hash_, command, kernel="void k_render<false, 0>(SceneView, MaskView"):
    with open(path, "w") as f:
        f.write("# rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE summary\n")
        f.write("# fetch command: %s\n# write command: %s\n" % (command, command))
        f.write("# source hash: %s\n" % hash_)
        f.write("kernel calls FETCH_KiB WRITE_KiB HBM_MB_scaled\n")
        f.write("%-72s %6d %16.1f %16.1f %14.2f\n" % (kernel, 1, 10.0, 5.0, 1234.5))


def test_counter_summaries_are_used_only_for_the_same_sources_and_rows(tmp_path, monkeypatch):
    """bench.py reports measured HBM bytes from a committed counter summary
    only when the summary's source hash is that of the HIP sources and its
    command rendered the rows the bench line renders."""
    sys.path.insert(0, ROOT)
    import bench
    import profile_summary
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setitem(bench.KERNELS, "render", "void k_render<false, 0>")
    (tmp_path / "profiles").mkdir()
    p = tmp_path / "profiles" / "render_blob1m_pmc.txt"
    cmd = "rocprofv3 --pmc FETCH_SIZE -- python3 bench.py --workload blob1m --rows 128"
    _summary(p, profile_summary.source_hash(), cmd)
    assert bench.profile_figures("blob1m", "render", 128) == {"traffic": int(1234.5 * 1e6)}
    assert bench.profile_figures("blob1m", "render", 0) == {}
    assert bench.profile_figures("blob1m", "render", 64) == {}
    _summary(p, "0" * 16, cmd)
    assert bench.profile_figures("blob1m", "render", 128) == {}
    _summary(p, profile_summary.source_hash(), cmd.replace(" --rows 128", ""))
    assert bench.profile_figures("blob1m", "render", 0) == {"traffic": int(1234.5 * 1e6)}
