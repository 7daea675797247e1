"""The oracle's own pins, run against builds of the oracle instrumented with
AddressSanitizer and UndefinedBehaviorSanitizer (host code only, gcc): any
out-of-bounds access, use after free, signed overflow or misaligned access in
the 2-D or 3-D oracle aborts the run. A planted one-element overrun shows that
the instrumentation is live.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC2 = os.path.join(ROOT, "oracle", "lbvp_ref.c")
SRC3 = os.path.join(ROOT, "oracle", "lbvp3_ref.c")
PINS = ["test_oracle_node.py", "test_oracle_grid.py", "test_oracle_moving.py", "test_oracle_step_nodes.py",
        "test_oracle3.py", "test_cuts.py"]

pytestmark = pytest.mark.slow


def _build(src, out):
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-o", out, src, "-lm"], check=True)


def _run_pins(lib2, lib3, log, files):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                          check=True).stdout.strip()
    env = dict(os.environ)
    # the sanitizer runtime must come first; whatever is preloaded already stays
    env["LD_PRELOAD"] = asan + (":" + env["LD_PRELOAD"] if env.get("LD_PRELOAD") else "")
    env.update(LBVP_REF_LIB=lib2, LBVP3_REF_LIB=lib3, OMP_NUM_THREADS="2",
               ASAN_OPTIONS=f"detect_leaks=0:log_path={log}", UBSAN_OPTIONS=f"print_stacktrace=1:log_path={log}")
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not slow"]
                          + [os.path.join(ROOT, "tests", f) for f in files],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=1500)


def _logs(tmp):
    return "".join(open(os.path.join(tmp, f)).read() for f in os.listdir(tmp) if f.startswith("san."))


def test_oracle_pins_clean_under_sanitizers():
    with tempfile.TemporaryDirectory() as tmp:
        lib2, lib3 = os.path.join(tmp, "ref2.so"), os.path.join(tmp, "ref3.so")
        _build(SRC2, lib2)
        _build(SRC3, lib3)
        r = _run_pins(lib2, lib3, os.path.join(tmp, "san"), PINS)
        logs = _logs(tmp)
        assert r.returncode == 0 and not logs, (r.stdout[-2000:], logs[:4000])


def test_sanitizers_catch_a_planted_overrun():
    src = open(SRC2).read()
    old = "for (int j = 0; j < ny; ++j) m += c->row_mass[j];"
    assert src.count(old) == 1
    with tempfile.TemporaryDirectory() as tmp:
        bad = os.path.join(tmp, "bad.c")
        with open(bad, "w") as f:
            f.write(src.replace(old, "for (int j = 0; j <= ny; ++j) m += c->row_mass[j];"))
        lib2, lib3 = os.path.join(tmp, "ref2.so"), os.path.join(tmp, "ref3.so")
        _build(bad, lib2)
        _build(SRC3, lib3)
        r = _run_pins(lib2, lib3, os.path.join(tmp, "san"), ["test_oracle_grid.py"])
        assert r.returncode != 0 and "heap-buffer-overflow" in _logs(tmp)
