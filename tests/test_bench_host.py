"""Host-side pieces of bench.py (CPU only): the eq. 4.1 term rule it uses for
the algorithmic byte model, the accumulator-update count, the hash that ties a
counter run to the kernel sources, and the one-GPU guard."""
import json
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("tol,terms", [(1e-3, 12), (1e-4, 16), (1e-6, 24), (1e-9, 35),
                                       (1e-10, 39), (1e-12, 47)])
def test_mass_rule_terms_is_eq_4_1(tol, terms):
    """Smallest M with 2 beta^(M+1)/(1+beta) <= tol at c = 0.85, the same as the
    oracle's own rule (written separately from Prop. 1 and eq. 4.1)."""
    assert bench.mass_rule_terms(0.85, tol) == terms
    assert oracle.terms_for_mass_error(0.85, tol) == terms


def test_acc_launches_by_hand():
    # 26 launches, first check at launch 24: groups of three start at launches
    # 0, 3, ..., 21 (8 groups, the last ending at 23), then the pair 24-25: 9
    assert bench.acc_launches(26, 24) == 9
    # no check before the first launch: pairs 0-1, 2-3, then the lone 4
    assert bench.acc_launches(5, 0) == 3
    assert bench.acc_launches(1, 0) == 1
    # every launch accounted for: the grouped count never exceeds the launches
    for n in range(1, 60):
        for k_min in (0, 5, 24, 80):
            assert (n + 2) // 3 <= bench.acc_launches(n, k_min) <= n


def test_code_only_drops_comments_and_keeps_literals():
    src = ('a = "x // y /* z */"; // line\n/* block\n more */ b = \'/\';\n'
           '  c = 1/2;   d = \'"\'; // end')
    assert bench.code_only(src) == 'a = "x // y /* z */"; b = \'/\'; c = 1/2; d = \'"\';'


def test_kernel_hash_ignores_comments_but_not_code(tmp_path):
    a = tmp_path / "a.hip"
    b = tmp_path / "b.hip"
    c = tmp_path / "c.hip"
    a.write_text("int f(int x) {\n  return x + 1;  // one\n}\n")
    b.write_text("/* the same code */ int f(int x)\n{ return x + 1; }\n")
    c.write_text("int f(int x) {\n  return x + 2;  // one\n}\n")
    assert bench.kernel_hash([str(a)]) == bench.kernel_hash([str(b)])
    assert bench.kernel_hash([str(a)]) != bench.kernel_hash([str(c)])


def test_load_traffic_needs_the_same_code_and_workload(tmp_path):
    src = tmp_path / "k.hip"
    src.write_text("int k;\n")
    t = tmp_path / "traffic.json"
    good = {"kernel_sha": bench.kernel_hash([str(src)]), "n": 10, "nnz": 20,
            "bytes_per_launch": 123.0}
    t.write_text(json.dumps(good))
    assert bench.load_traffic(10, 20, str(t), [str(src)]) == 123.0
    assert bench.load_traffic(11, 20, str(t), [str(src)]) is None
    assert bench.load_traffic(10, 21, str(t), [str(src)]) is None
    src.write_text("int k2;\n")
    assert bench.load_traffic(10, 20, str(t), [str(src)]) is None
    assert bench.load_traffic(10, 20, str(tmp_path / "missing.json"), [str(src)]) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_cpu_baselines_of_the_secondary_workloads():
    """The per-workload CPU baselines run the C oracle on a sample of the same
    workload: single sources with a given term count, and graphs cut out of a
    block-diagonal batch (local labels, their own term counts)."""
    import graphgen as gg
    g = gg.chung_lu(3000, 8, 2.3, seed=3)
    r = bench.cpu_baseline_sources(g, 0.85, [0, 5], 10)
    assert r["kind"] == "oracle" and r["unit"] == "GTEPS" and r["value"] > 0
    assert r["solves_per_s"] > 0 and r["cores"] >= 1
    r = bench.cpu_baseline_sources(g, 0.85, [0], 10, unit="solves/s")
    assert r["value"] == r["solves_per_s"]
    batch = gg.uneven_batch(12, seed=5)
    _, p = gg.batch_sources(batch, seed=5)
    terms = [20] * batch.num_graphs
    r = bench.cpu_baseline_graphs(batch, 0.85, p, terms, sample=5)
    assert r["value"] > 0 and "first 5 graphs" in r["sample"]


def test_emit_prints_the_line_when_the_copy_cannot_run(capsys, monkeypatch):
    """The copy bandwidth is context added after the timed region: when it
    cannot be measured the line is printed as it was, and when it can the
    fraction is achieved over the copy's rate."""
    def no_gpu():
        raise RuntimeError("no device")
    monkeypatch.setattr(bench, "copy_bandwidth", no_gpu)
    line = {"value": 1.0, "roofline": {"unit": "GB/s", "achieved": 10.0}}
    bench.emit(dict(line, roofline=dict(line["roofline"])))
    assert json.loads(capsys.readouterr().out) == line
    monkeypatch.setattr(bench, "copy_bandwidth", lambda: 40.0)
    bench.emit(dict(line, roofline=dict(line["roofline"])))
    rf = json.loads(capsys.readouterr().out)["roofline"]
    assert rf["copy_gbs"] == 40.0 and rf["frac_of_copy"] == 0.25
    # a roofline in other units (TFLOP/s) gets no copy figure
    bench.emit({"value": 1.0, "roofline": {"unit": "TFLOP/s", "achieved": 1.0}})
    assert "copy_gbs" not in json.loads(capsys.readouterr().out)["roofline"]
