"""bench.py reports a kernel's HBM traffic only while the committed counter
summaries were taken on the sources that run: its source hash must cover
every header the hashed sources include from the kernel directory, or an
edit there would leave stale counters in the bench line."""
import importlib.util
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2501_05244_amd", "csrc")


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_source_hash_covers_included_headers():
    names = set(_bench().KERNEL_SOURCES)
    seen, todo = set(), list(names)
    while todo:
        name = todo.pop()
        if name in seen:
            continue
        seen.add(name)
        with open(os.path.join(CSRC, name)) as fh:
            for inc in re.findall(r'^\s*#include\s+"([^"]+)"', fh.read(), re.M):
                if os.path.exists(os.path.join(CSRC, inc)):
                    assert inc in names, f"{name} includes {inc}, which the source hash does not cover"
                    todo.append(inc)


def test_source_hash_changes_with_any_hashed_source(tmp_path):
    import shutil
    b = _bench()
    dst = tmp_path / "paper_2501_05244_amd" / "csrc"
    dst.mkdir(parents=True)
    for name in b.KERNEL_SOURCES:
        shutil.copy(os.path.join(CSRC, name), dst / name)
    b.ROOT = str(tmp_path)
    h0 = b.kernel_source_hash()
    assert len(h0) == 64 and h0 == b.kernel_source_hash()
    for name in b.KERNEL_SOURCES:
        f = dst / name
        text = f.read_text()
        f.write_text(text + "\n// edited\n")
        assert b.kernel_source_hash() != h0, name
        f.write_text(text)
    assert b.kernel_source_hash() == h0
