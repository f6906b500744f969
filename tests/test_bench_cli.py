"""bench.py on the CPU: the one-GPU contract and the source hash that keys
measured traffic to the kernel code it was taken on."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_source_hash_ignores_comments_but_not_code(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2003_02256_amd" / "csrc"
    csrc.mkdir(parents=True)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    code = "int f(int x) {\n  return x + 1;\n}\n"

    def h(text):
        (csrc / "k.hip").write_text(text)
        return bench.kernel_source_hash(["k.hip"])

    base = h(code)
    assert h("// a header\n" + code.replace("x + 1;", "x + 1;  // one more")) == base
    assert h("/* block\n comment */\n" + code + "\n\n") == base
    assert h(code.replace("x + 1", "x + 2")) != base
