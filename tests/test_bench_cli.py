"""Host logic of bench.py (no GPU): argument checks that end the run before
any device call, and the algorithmic byte model the roofline fractions
divide by."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_byte_model():
    """Values per cell: flux stage 1 reads U and Sigma and writes U (11),
    stages 2 and 3 also read U^n (16); the stress reads rho and m and writes
    six components; the viscous flux divergence reads rho, m and the six
    components and reads and writes four output fields."""
    assert bench.algorithmic_bytes_per_cell("flux_rk", "f64", 10) == 8 * (11 + 16 + 16) / 3
    assert bench.algorithmic_bytes_per_cell("flux_rk", "f32", 10) == 4 * (11 + 16 + 16) / 3
    assert bench.algorithmic_bytes_per_cell("stress", "f64", 10) == 8 * 10
    assert bench.algorithmic_bytes_per_cell("stress", "f32", 10) == 4 * 10
    assert bench.algorithmic_bytes_per_cell("viscous", "f64", 10) == 8 * 18
    assert bench.algorithmic_bytes_per_cell("viscous", "f32", 10) == 4 * 18
    # split form: FP32 U^n, BF16 differences; rho, m of stages 2 and 3 read
    # both, the outputs of stages 1 and 2 are differences
    assert bench.algorithmic_bytes_per_cell("stress", "bf16d", 10) == 4 * (4 + 2 * 2 / 3) + 6 * 4
    assert bench.algorithmic_bytes_per_cell("viscous", "bf16d", 10) == 4 * (4 + 2 * 2 / 3) + 6 * 4 + (2 * 16 + 32) / 3
    with pytest.raises(KeyError):
        bench.algorithmic_bytes_per_cell("nonesuch", "f64", 10)


def test_sigma_schedule_counts_the_launches_of_a_solve():
    """(source-forming passes, later two-sweep passes, later single sweeps)
    per solve, as the library launches them: an even Jacobi count with
    two-sweep passes starts with a two-sweep first pass, an odd one with a
    single first sweep; red-black runs one pass per sweep with two-level
    passes, else two half-sweep launches per sweep."""
    assert bench.sigma_schedule(10, 2) == (1, 4, 0)
    assert bench.sigma_schedule(5, 2) == (1, 2, 0)
    assert bench.sigma_schedule(5, 1) == (1, 0, 4)
    assert bench.sigma_schedule(0, 2) == (0, 0, 0)
    assert bench.sigma_schedule(10, 2, "rbgs") == (1, 9, 0)
    assert bench.sigma_schedule(10, 1, "rbgs") == (1, 0, 19)
    # FP64 Jacobi bytes per launch at S = 10: (56 + 4 x 32) / 5 per cell
    assert bench.algorithmic_bytes_per_cell("jacobi", "f64", 10, 2) == (56 + 4 * 32) / 5
    assert bench.algorithmic_bytes_per_cell("jacobi", "f64", 10, 2, "rbgs") == (56 + 9 * 32) / 10
    # with viscous terms the first pass also writes the stress
    assert bench.algorithmic_bytes_per_cell("jacobi", "f64", 10, 2, viscous=True) == (56 + 48 + 4 * 32) / 5
    assert bench.algorithmic_bytes_per_cell("jacobi", "f64", 5, 2, viscous=True) == (56 + 48 + 2 * 32) / 3
    assert bench.algorithmic_bytes_per_cell("jacobi", "f64", 10, 1, viscous=True) == (56 + 48 + 9 * 32) / 10


def test_rooflines_skip_kernels_that_did_not_run():
    kt = {"flux_rk": (84.0, 2), "jacobi": (0.0, 0), "stress": (0.0, 0), "viscous": (0.0, 0)}
    r = bench.kernel_rooflines(kt, 1000, "f64", 10, 2)
    assert set(r) == {"flux_rk"}
    gbs = bench.algorithmic_bytes_per_cell("flux_rk", "f64", 10) * 1000 / (42.0e-3) / 1e9
    assert r["flux_rk"]["achieved_GBs"] == round(gbs, 1)
    assert r["flux_rk"]["frac"] == round(gbs / bench.HBM_PEAK_GBS, 4)


def test_source_hash_ignores_comments_only():
    """The counter summaries are tied to the kernel code: comments and
    layout do not change the hash, code does (string literals are code)."""
    a = 'int f(int x) { return x + 1; }  // one\n/* two */ const char* s = "// not a comment";\n'
    b = '// header\nint f(int x)\n{\n    return x + 1;   /* same */\n}\nconst char* s = "// not a comment";\n'
    c = 'int f(int x) { return x + 2; }\nconst char* s = "// not a comment";\n'
    d = 'int f(int x) { return x + 1; }\nconst char* s = "// a comment?";\n'
    assert bench.strip_comments(a) == bench.strip_comments(b)
    assert bench.strip_comments(a) != bench.strip_comments(c)
    assert bench.strip_comments(a) != bench.strip_comments(d)
    assert len(bench.kernel_source_hash()) == 16
