"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

Its C source is built with gcc -fsanitize=address,undefined (every finding
fatal) and the oracle pin suite (tests/test_oracle.py) runs against that
build in a child process, with the ASan runtime preloaded (the Python
interpreter itself is not instrumented).  An out-of-bounds access, a use
after free, a signed overflow or a misaligned access anywhere the pins reach
ends the child with the sanitizer's report instead of a pass.  CPU only.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "dibella_oracle.c")

# capture=sys: the sanitizers write their reports to file descriptor 2,
# which must reach the parent even when the child dies mid-test
_CHILD = (
    "import sys, pytest, oracle\n"
    "oracle.use_library(sys.argv[1])\n"
    "sys.exit(pytest.main([sys.argv[2], '-x', '-q', '--capture=sys', '-p', 'no:cacheprovider', '-m', 'not gpu']))\n"
)


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _sanitized_build(tmp_path, extra=()):
    so = str(tmp_path / "oracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c99", "-fPIC", "-shared", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", *extra,
                           "-o", so, SRC])
    return so


def _run(so, target):
    asan = _runtime("libasan.so")
    pre = " ".join(p for p in (asan, os.environ.get("LD_PRELOAD", "")) if p)
    env = dict(os.environ, PYTHONDONTWRITEBYTECODE="1", OMP_NUM_THREADS="1", PYTHONPATH=ROOT, LD_PRELOAD=pre,
               # the interpreter's own allocations are not the oracle's: no leak report
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:exitcode=23",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1:exitcode=24")
    return subprocess.run([sys.executable, "-c", _CHILD, so, target], cwd=ROOT, env=env,
                          capture_output=True, text=True, timeout=1200)


@pytest.mark.skipif(_runtime("libasan.so") is None or _runtime("libubsan.so") is None,
                    reason="gcc's sanitizer runtimes are not installed")
def test_oracle_pins_pass_under_asan_and_ubsan(tmp_path):
    so = _sanitized_build(tmp_path)
    r = _run(so, os.path.join("tests", "test_oracle.py"))
    out = r.stdout[-3000:] + r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out
    assert r.returncode == 0, out


@pytest.mark.skipif(_runtime("libasan.so") is None, reason="gcc's sanitizer runtimes are not installed")
def test_the_sanitized_build_reports_an_out_of_bounds_read(tmp_path):
    """The set-up itself works: a build with a planted one-past-the-end read
    in the transpose fails under ASan with its report."""
    with open(SRC) as f:
        text = f.read()
    old = "memcpy(fill, t_rowptr, sizeof(int64_t) * (size_t)(m + 1));"
    assert old in text, "the planted read needs the transpose's fill array"
    planted = text.replace(old, old + "\n    { volatile int64_t past = fill[m + 1]; (void)past; }", 1)
    c = tmp_path / "planted.c"
    c.write_text(planted)
    so = str(tmp_path / "planted.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c99", "-fPIC", "-shared", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", so, str(c)])
    r = _run(so, os.path.join("tests", "test_oracle.py") + "::test_transpose_lists_each_column_by_read")
    assert r.returncode != 0 and "AddressSanitizer" in (r.stdout + r.stderr), r.stdout[-2000:] + r.stderr[-2000:]
