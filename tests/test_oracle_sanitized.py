"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer runs
its hand-derived and small-input pins cleanly (CPU only).

A sanitized copy of oracle/tpc_oracle.c is compiled with gcc, and the pins
run in a child Python process that preloads the ASan runtime and loads that
copy (TPC_ORACLE_LIB); any out-of-bounds access, use after free, signed
overflow or other undefined behaviour aborts the child and fails the test.
"""
import os
import subprocess
import sys

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

PINS = ("golden_neighbour_rule or score_weights_decide or grid_structure or y_cells or lexsort or "
        "bruteforce_tiny or whole_row_mode or invariant_under_bin or true_neighbours or chain_invariants or "
        "propagation or jacobian or seed_exact or noise_free_helix or agrees_with_two_pass or "
        "pickup_score or pickup_tie or max_miss or keep_threshold or leaves_the_sector or fragile_flag or "
        "owner_is_max or invalid_inputs or empty_and_sparse or zero_field")


def _sanitized_run(tmp_path, src_text, pins):
    src = tmp_path / "oracle_san.c"
    src.write_text(src_text)
    lib = tmp_path / "oracle_san.so"
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-fopenmp", "-std=c11", "-D_POSIX_C_SOURCE=200809L",
                           "-shared", "-fPIC", "-o", str(lib), str(src), "-lm"])
    asan_rt = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    assert os.path.isabs(asan_rt), "no ASan runtime for gcc"
    env = dict(os.environ, TPC_ORACLE_LIB=str(lib), LD_PRELOAD=asan_rt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")
    probe = subprocess.run([sys.executable, "-c", "import oracle; oracle._load(); print(oracle._LIB)"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert probe.returncode == 0 and probe.stdout.strip() == str(lib), probe.stdout + probe.stderr
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-s", "-p", "no:cacheprovider", "-p", "no:xdist",
                           os.path.join(HERE, "test_oracle_pins.py"), "-k", pins],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)


def test_pins_under_sanitizers(tmp_path):
    r = _sanitized_run(tmp_path, open(oracle._SRC).read(), PINS)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert " passed" in r.stdout and "ERROR: AddressSanitizer" not in r.stderr, tail
    assert "runtime error" not in r.stderr, tail


def test_sanitizers_catch_a_planted_overflow(tmp_path):
    """The harness is live: a copy that clears one entry past each tracklet's
    hit row (the last one runs off its allocation) fails under ASan."""
    src = open(oracle._SRC).read()
    find = "for (int64_t r = 0; r < R; ++r) t->hits[r] = -1;"
    assert src.count(find) == 1
    r = _sanitized_run(tmp_path, src.replace(find, "for (int64_t r = 0; r <= R; ++r) t->hits[r] = -1;"),
                       "keep_threshold")
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr, (r.stdout + r.stderr)[-2000:]
