"""Host-side checks of bench.py's bookkeeping (no GPU): the HBM traffic read from the
committed byte-counter summary is reported only while the counted kernel's source is the
one the counters were taken on."""
import hashlib
import importlib.util
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture()
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _tree(tmp_path, src_text, digest, kernel="sketch_pass_bf16", nbytes=1234567, file_kernel="sketch_pass_bf16"):
    src = tmp_path / "k.hip"
    src.write_text(src_text)
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / f"hbm_counters_{file_kernel}_1024x1024x512.md").write_text(
        "summary text\n\n"
        f"traffic_kernel: {kernel}\n"
        f"traffic_bytes_per_launch: {nbytes}\n"
        f"source_sha256(k.hip): {digest}\n")
    return src


def test_traffic_reported_while_source_matches(bench, tmp_path, monkeypatch):
    text = "kernel source\n"
    _tree(tmp_path, text, hashlib.sha256(text.encode()).hexdigest())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counter_traffic("sketch_pass_bf16") == 1234567


def test_traffic_withheld_once_source_changes(bench, tmp_path, monkeypatch):
    text = "kernel source\n"
    src = _tree(tmp_path, text, hashlib.sha256(text.encode()).hexdigest())
    src.write_text(text + "// edited\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counter_traffic("sketch_pass_bf16") is None


def test_traffic_withheld_for_another_kernel(bench, tmp_path, monkeypatch):
    text = "kernel source\n"
    _tree(tmp_path, text, hashlib.sha256(text.encode()).hexdigest())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counter_traffic("core_ttm1_bf16") is None


def test_traffic_withheld_when_summary_names_another_kernel(bench, tmp_path, monkeypatch):
    text = "kernel source\n"
    _tree(tmp_path, text, hashlib.sha256(text.encode()).hexdigest(), kernel="sketch_pass_bf16",
          file_kernel="core_ttm1_f32")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counter_traffic("core_ttm1_f32") is None


def test_traffic_withheld_without_summary(bench, tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counter_traffic("sketch_pass_bf16") is None


@pytest.mark.parametrize("path", sorted(p for p in os.listdir(os.path.join(ROOT, "profiles"))
                                        if p.startswith("hbm_counters_") and p.endswith("_1024x1024x512.md")))
def test_committed_summary_is_well_formed(bench, path):
    # each committed summary names its kernel, a positive byte count and a source file that
    # exists; whether its hash still matches depends on later edits and is not asserted
    text = open(os.path.join(ROOT, "profiles", path)).read()
    kernel = path[len("hbm_counters_"):-len("_1024x1024x512.md")]
    assert re.search(rf"^traffic_kernel: {kernel}$", text, re.M)
    m = re.search(r"^traffic_bytes_per_launch: (\d+)$", text, re.M)
    assert m and int(m.group(1)) > 0
    m = re.search(r"^source_sha256\((\S+)\): [0-9a-f]{64}$", text, re.M)
    assert m and os.path.exists(os.path.join(ROOT, m.group(1)))


def test_bench_calls_only_existing_binding_functions():
    """Every rt.<name> that bench.py and the GPU tests call exists in the binding (a missing one
    would only show on the GPU machine)."""
    import paper_2211_13028_amd as rt
    names = set()
    for path in [os.path.join(ROOT, "bench.py"), os.path.join(ROOT, "__graft_entry__.py")] + [
            os.path.join(ROOT, "tests", f) for f in os.listdir(os.path.join(ROOT, "tests")) if f.endswith(".py")]:
        names |= set(re.findall(r"\brt\.(rtucker_\w+|Batch|NOALLOC_\w+)", open(path).read()))
    missing = sorted(n for n in names if not hasattr(rt, n))
    assert not missing, missing
