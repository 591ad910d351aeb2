"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of the oracle source (a dropped term,
a wrong comparison, a swapped operand, a wrong index or order), builds it,
and runs the oracle pin suite (tests/test_oracle.py) against it in a child
process: the suite must fail.  The unedited source, built the same way, must
pass.  Everything here runs on the CPU.
"""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "dibella_oracle.c")

# (id, text in the oracle source, replacement); the first occurrence is edited
MUTANTS = [
    # overlap: add (count, seeds) and the order of k
    ("seed-keeps-one", "if (c < 2) {", "if (c < 1) {"),
    ("seed-pair-swapped", "seeds[4 * j + 2 * c + 0] = val[e];\n                    seeds[4 * j + 2 * c + 1] = t_pos[f];",
     "seeds[4 * j + 2 * c + 0] = t_pos[f];\n                    seeds[4 * j + 2 * c + 1] = val[e];"),
    ("min-shared-strict", "if (count[j] >= min_shared) {", "if (count[j] > min_shared) {"),
    ("diagonal-dropped", "int32_t j = t_read[f];\n                if (count[j] == 0) {",
     "int32_t j = t_read[f];\n                if (j == (int32_t)i) continue;\n                if (count[j] == 0) {"),
    ("k-walked-descending", "for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {\n            int32_t k = col[e];\n            for (int64_t f = t_rowptr[k];",
     "for (int64_t e = rowptr[i + 1] - 1; e >= rowptr[i]; --e) {\n            int32_t k = col[e];\n            for (int64_t f = t_rowptr[k];"),
    ("count-double", "int32_t c = count[j]++;", "int32_t c = count[j]; count[j] += 2;"),
    # reduction: the MinPlus semiring
    ("walk-check-inverted", "if (dst_of(r_ik) != src_of(r_kj)) return INF_KEY;", "if (dst_of(r_ik) == src_of(r_kj)) return INF_KEY;"),
    ("walk-check-wrong-heads", "if (dst_of(r_ik) != src_of(r_kj)) return INF_KEY;", "if (src_of(r_ik) != dst_of(r_kj)) return INF_KEY;"),
    ("sum-drops-term", "uint32_t sum = (uint32_t)(oh_of(r_ik) + oh_of(r_kj));", "uint32_t sum = (uint32_t)(oh_of(r_kj));"),
    ("end-code-swapped", "return (sum << 2) | (uint32_t)(src_of(r_ik) << 1) | (uint32_t)dst_of(r_kj);",
     "return (sum << 2) | (uint32_t)(dst_of(r_kj) << 1) | (uint32_t)src_of(r_ik);"),
    ("add-is-max", "static uint32_t minplus_add(uint32_t a, uint32_t b) { return a < b ? a : b; }",
     "static uint32_t minplus_add(uint32_t a, uint32_t b) { return (a == INF_KEY) ? b : (b == INF_KEY ? a : (a > b ? a : b)); }"),
    # reduction: v, M, I and the loop
    ("row-max-is-first", "if (oh_of(va[e]) > v[i]) v[i] = oh_of(va[e]);", "if (v[i] == 0) v[i] = oh_of(va[e]);"),
    ("fuzz-not-added", "if (v[i] != 0) v[i] += fuzz;", "if (v[i] != 0) v[i] += 0;"),
    ("edge-rule-no-fuzz", "(int64_t)oh_of(va[e]) + fuzz : (int64_t)v[i];", "(int64_t)oh_of(va[e]) : (int64_t)v[i];"),
    ("compare-strict", "(int64_t)(nij >> 2) <= mij;", "(int64_t)(nij >> 2) < mij;"),
    ("end-check-dropped", "int transitive = nij != INF_KEY && (int32_t)(nij & 3u) == code_of(va[e]) &&",
     "int transitive = nij != INF_KEY &&"),
    ("contained-kept", "if (oh_of(val[e]) > 0) { ci[nnz] = col[e];", "if (oh_of(val[e]) >= 0) { ci[nnz] = col[e];"),
    ("one-pass-only", "} while (nnz != prev);", "} while (0);"),
    ("variant-b-inverted", "(rcode[j] < 0 || (int32_t)(key & 3u) != rcode[j])", "(rcode[j] < 0 || (int32_t)(key & 3u) == rcode[j])"),
    # overlap graph from the seeds of C
    ("rfs-strand-ignored", "*rc = (a & 1) != (b & 1);", "*rc = 0;"),
    ("rfs-rc-offset", "return *rc ? pi + pj + k - lj : pi - pj;", "return *rc ? pi + pj - lj : pi - pj;"),
    ("rfs-offset-sign", "return *rc ? pi + pj + k - lj : pi - pj;", "return *rc ? pi + pj + k - lj : pj - pi;"),
    ("rfs-inner-code", "code = rc ? 1 : 0;                       /* (0,0) or (0,1) */",
     "code = rc ? 2 : 0;                       /* (0,0) or (0,1) */"),
    ("rfs-outer-code", "code = rc ? 2 : 3;                       /* (1,0) or (1,1) */",
     "code = rc ? 1 : 3;                       /* (1,0) or (1,1) */"),
    ("rfs-suffix-past", "suffix = d + lj - li;", "suffix = d + lj;"),
    ("rfs-suffix-before", "suffix = -d;", "suffix = li - d - lj;"),
    ("rfs-contained-kept", "if (overlap == li || overlap == lj) {", "if (0) {"),
    ("rfs-min-overlap-strict", "if (overlap < min_overlap) continue;", "if (overlap <= min_overlap) continue;"),
    ("rfs-second-seed", "int32_t a = c_seed[4 * e + 0], b = c_seed[4 * e + 1];",
     "int32_t a = c_seed[4 * e + 1], b = c_seed[4 * e + 0];"),
    ("rfs-drift-unchecked", "if (rc1 != rc || d1 - d > max_drift || d - d1 > max_drift) continue;",
     "if (rc1 != rc) continue;"),
    ("rfs-drift-orientation-ignored", "if (rc1 != rc || d1 - d > max_drift || d - d1 > max_drift) continue;",
     "if (d1 - d > max_drift || d - d1 > max_drift) continue;"),
    ("rfs-drift-strict", "if (rc1 != rc || d1 - d > max_drift || d - d1 > max_drift) continue;",
     "if (rc1 != rc || d1 - d >= max_drift || d - d1 >= max_drift) continue;"),
    ("rfs-no-second-seed-kept", "if (a1 < 0 || b1 < 0) continue;", "if (a1 < 0 || b1 < 0) a1 = a, b1 = b;"),
    ("rfs-density-unchecked", "if (min_density > 0 && (int64_t)c_count[e] * 10000 < (int64_t)min_density * overlap) continue;",
     "if (0) continue;"),
    ("rfs-density-strict", "if (min_density > 0 && (int64_t)c_count[e] * 10000 < (int64_t)min_density * overlap) continue;",
     "if (min_density > 0 && (int64_t)c_count[e] * 10000 <= (int64_t)min_density * overlap) continue;"),
    ("rfs-density-per-kbp", "if (min_density > 0 && (int64_t)c_count[e] * 10000 < (int64_t)min_density * overlap) continue;",
     "if (min_density > 0 && (int64_t)c_count[e] * 1000 < (int64_t)min_density * overlap) continue;"),
    # A from the reads
    ("km-strand-inverted", "win[w].strand = rc < fwd;", "win[w].strand = rc > fwd;"),
    ("km-not-canonical", "win[w].code = rc < fwd ? rc : fwd;", "win[w].code = fwd;"),
    ("km-rc-not-reversed", "rc |= (uint64_t)(3 - s[p + q]) << (2 * q);", "rc = (rc << 2) | (uint64_t)(3 - s[p + q]);"),
    ("km-rc-not-complemented", "rc |= (uint64_t)(3 - s[p + q]) << (2 * q);", "rc |= (uint64_t)s[p + q] << (2 * q);"),
    ("km-bounds-strict", "if (freq >= lo && freq <= hi) {", "if (freq > lo && freq <= hi) {"),
    ("km-upper-bound-dropped", "if (freq >= lo && freq <= hi) {", "if (freq >= lo) {"),
    ("km-last-position", "if (e > runs[c].a && win[e].read == win[e - 1].read) continue;",
     "if (e + 1 < runs[c].b && win[e].read == win[e + 1].read) continue;"),
    ("km-columns-in-code-order", "qsort(runs, (size_t)m, sizeof(oracle_run), cmp_run_first);", ""),
    ("km-first-occurrence-last-position", "return (p->pos > q->pos) - (p->pos < q->pos);",
     "return (p->pos < q->pos) - (p->pos > q->pos);"),
    ("km-last-base-first", "fwd = (fwd << 2) | s[p + q];", "fwd |= (uint64_t)s[p + q] << (2 * q);"),
    ("km-window-past-end", "for (int64_t p = 0; p + k <= L; ++p) {", "for (int64_t p = 0; p + k < L; ++p) {"),
    # one-pass marks used for sampled checks
    ("marks-compare-strict", "(int64_t)(nij >> 2) <= mij);", "(int64_t)(nij >> 2) < mij);"),
    ("marks-row-max-unset", "if (vi != 0) vi += fuzz;", "if (vi != 0) vi += fuzz + 1;"),
    # X-drop extension and R from the alignment
    ("xd-drop-strict", "if (v != ORACLE_XD_DEAD && v < best - X) v = ORACLE_XD_DEAD;",
     "if (v != ORACLE_XD_DEAD && v <= best - X) v = ORACLE_XD_DEAD;"),
    ("xd-last-max-in-diagonal", "if (v > dbest) { dbest = v; di = i; }", "if (v >= dbest) { dbest = v; di = i; }"),
    ("xd-later-diagonal-ties", "if (dbest != ORACLE_XD_DEAD && dbest > best)", "if (dbest != ORACLE_XD_DEAD && dbest >= best)"),
    ("xd-match-inverted", "(a[i - 1] == b[j - 1] ? mat : mis)", "(a[i - 1] != b[j - 1] ? mat : mis)"),
    ("xd-one-gap-direction", "if (j >= 1 && dg[1][i] != ORACLE_XD_DEAD", "if (0 && j >= 1 && dg[1][i] != ORACLE_XD_DEAD"),
    ("xd-one-dead-diagonal-stops", "if (lo[0] > hi[0] && lo[1] > hi[1]) {", "if (lo[1] > hi[1]) {"),
    ("xd-band-off-by-one", "if (to - from + 1 > ORACLE_XD_BAND) break;", "if (to - from + 1 >= ORACLE_XD_BAND) break;"),
    ("al-rc-position-unflipped", "q = rc ? lj - k - (b >> 1) : (b >> 1);", "q = (b >> 1);"),
    ("al-j-not-complemented", "return rc ? (uint8_t)(3 - s[L - 1 - x]) : s[x];", "return rc ? s[L - 1 - x] : s[x];"),
    ("al-left-not-reversed", "for (int64_t x = 0; x < ml; ++x) al[x] = si[pi - 1 - x];",
     "for (int64_t x = 0; x < ml; ++x) al[x] = si[x];"),
    ("al-score-without-seed", "int64_t score = sl + (int64_t)k * mat + sr;", "int64_t score = sl + sr;"),
    ("al-min-score-strict", "if (score < min_score) continue;", "if (score <= min_score) continue;"),
    ("al-contained-one-way", "if ((bj >= bi && rj >= ri) || (bi >= bj && ri >= rj)) {", "if (bj >= bi && rj >= ri) {"),
    ("al-suffix-past", "val = (int32_t)(((rj - ri) << 2) | (rc ? 1 : 0));", "val = (int32_t)((rj << 2) | (rc ? 1 : 0));"),
    ("al-ends-swapped", "int64_t bi = pi - eal, ei = pi + k + ear, bj = q - ebl, ej = q + k + ebr;",
     "int64_t bi = pi - ebl, ei = pi + k + ear, bj = q - eal, ej = q + k + ebr;"),
]


def _build(text, out_dir, name):
    c = os.path.join(out_dir, name + ".c")
    so = os.path.join(out_dir, name + ".so")
    with open(c, "w") as f:
        f.write(text)
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-o", so, c])
    return so


# The child loads the planted build explicitly (oracle.use_library) before
# running the pins in-process: no environment variable swaps the oracle.
_CHILD = (
    "import sys, pytest, oracle\n"
    "oracle.use_library(sys.argv[1])\n"
    "sys.exit(pytest.main([sys.argv[2], '-x', '-q', '-p', 'no:cacheprovider', '-m', 'not gpu']))\n"
)


def _run_pins(so):
    # one thread per child: the children run side by side
    env = dict(os.environ, PYTHONDONTWRITEBYTECODE="1", OMP_NUM_THREADS="1", MKL_NUM_THREADS="1",
               OPENBLAS_NUM_THREADS="1", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", _CHILD, so, os.path.join("tests", "test_oracle.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout[-3000:] + r.stderr[-2000:]


def _all_outcomes(d):
    """Build the control and every planted copy in `d`, then run the pin
    suite against each of them, several child processes at a time."""
    from concurrent.futures import ThreadPoolExecutor
    with open(SRC) as f:
        text = f.read()
    jobs = {"control": text}
    for mid, old, new in MUTANTS:
        jobs[mid] = text.replace(old, new, 1) if old in text else None
    libs = {mid: (_build(src, d, mid) if src is not None else None) for mid, src in jobs.items()}
    workers = max(1, min(8, (os.cpu_count() or 2) // 2))
    with ThreadPoolExecutor(workers) as ex:
        futs = {mid: ex.submit(_run_pins, so) for mid, so in libs.items() if so}
        return {mid: f.result() for mid, f in futs.items()}


@pytest.fixture(scope="module")
def outcomes(tmp_path_factory):
    """The pin suite's outcome on the control and on every planted copy.
    Under pytest-xdist the first worker to get here computes them and the
    others read its file (the temporary root's parent is shared by the
    workers), so the suite runs once per session, not once per worker."""
    if not os.environ.get("PYTEST_XDIST_WORKER"):
        return _all_outcomes(str(tmp_path_factory.mktemp("oracle_mutants")))
    from filelock import FileLock
    shared = tmp_path_factory.getbasetemp().parent
    path = shared / "oracle_mutants.json"
    with FileLock(str(path) + ".lock"):
        if path.is_file():
            return json.loads(path.read_text())
        res = _all_outcomes(str(tmp_path_factory.mktemp("oracle_mutants")))
        path.write_text(json.dumps(res))
        return res


def test_unedited_oracle_passes_the_pins(outcomes):
    rc, out = outcomes["control"]
    assert rc == 0, out


@pytest.mark.parametrize("mid,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(outcomes, mid, old, new):
    assert mid in outcomes, f"{mid}: the text to edit is not in the oracle source"
    rc, out = outcomes[mid]
    # a failing assertion, not a crash or a collection error
    assert rc == 1 and " failed" in out, f"{mid}: the pins did not catch it (rc {rc})\n{out}"
