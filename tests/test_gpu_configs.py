"""The named workloads at their full sizes, through the C ABI, against the
oracle on sampled outputs.

Every case runs the library once at the workload's full shape and storage,
then checks, for a sample of rows of op(A) and columns of op(B): the shifts
log2 mu_i, log2 nu_j of those lines (they depend on the whole bound product,
which the oracle forms only for the sampled lines, ref.line_bounds), every
sampled output bit for bit against the oracle, and the normalised error
max |C - AB| / (|A||B|) against a double-double reference on the rows and
columns the accuracy sweep (accuracy_sweep) measures.  The sample is those
rows (first, middle, last, five seeded) and the first 128 or 512 of its 1024
columns, plus edge and seeded lines on both sides (the error of a subset of
the sweep's sample is at most the sweep's).  The number of moduli of each case is
the smallest that reached 1e-15 in the sweeps recorded under profiles/
(accuracy_sweep_*.md); the error bound is asserted at that count.

  * square workloads m = n = k in {4096, 8192}, phi in {0.5, 2, 4} (the
    paper's accuracy experiment, Section V-A; 8192^3 at phi = 0.5 is the
    benchmark workload, tested in test_gpu_parity.py);
  * rectangular workloads (1024, 1024, 65536) and (16384, 16384, 1024),
    phi = 1, all four transA / transB combinations (Sections V-B, V-C);
  * the large stress workload 16384^3 with a cancellation block: accurate
    mode at phi = 1 (12 moduli), and phi = 6 through the FP8 hybrid path and
    the INT8 arm at equal accuracy (20 and 24 moduli, both 2.2e-16 in the
    sweep).
"""
import numpy as np
import pytest

from gpu_util import check_sampled, sample_lines, sweep_sample
from workloads import cancellation_block, phi_matrix, phi_seed

pytestmark = pytest.mark.gpu


def _samples(m, n, seed, ncols=1024, cancel=False, extra=()):
    """The sweep's rows and its first `ncols` columns (the error is taken
    there: a subset of the sweep's sample, so its error bound carries over),
    plus edge and seeded lines for the bit-exact comparison."""
    er, ec = sweep_sample(m, n, cancel)
    ec = ec[:ncols]
    rows = np.union1d(er, sample_lines(m, 16, seed, extra))
    cols = np.union1d(ec, sample_lines(n, 16, seed + 1, extra))
    return rows, cols, er, ec


# ---- square workloads ----

SQUARE = [(4096, 0.5, 12), (4096, 2.0, 14), (4096, 4.0, 17), (8192, 2.0, 13), (8192, 4.0, 16)]


@pytest.mark.parametrize("size,phi,N", SQUARE)
def test_square_workloads(size, phi, N):
    label = f"square {size} phi={phi}"
    print(f"{label}: generating", flush=True)
    s = phi_seed(2, phi)
    A = phi_matrix(size, size, phi, s)
    B = phi_matrix(size, size, phi, s + 1)
    rows, cols, er, ec = _samples(size, size, 100 + size, ncols=512)
    check_sampled(A, B, N, rows, cols, err_rows=er, err_cols=ec, label=label)


# ---- rectangular workloads, all four storage orders ----

RECT = [(1024, 1024, 65536), (16384, 16384, 1024)]
RECT_N = 12


@pytest.fixture(scope="module")
def rect_inputs():
    held = {}

    def get(shape):
        if shape not in held:
            held.clear()
            m, n, k = shape
            s = phi_seed(3, 1.0)
            print(f"rect {shape}: generating", flush=True)
            A = phi_matrix(m, k, 1.0, s)
            B = phi_matrix(k, n, 1.0, s + 1)
            held[shape] = (A, B, _samples(m, n, 300 + m, ncols=128 if k > 8192 else 512), {})
        return held[shape]

    yield get
    held.clear()


@pytest.mark.parametrize("shape", RECT)
@pytest.mark.parametrize("ta,tb", [("N", "N"), ("T", "N"), ("N", "T"), ("T", "T")])
def test_rectangular_workloads(rect_inputs, shape, ta, tb):
    A, B, (rows, cols, er, ec), cache = rect_inputs(shape)
    check_sampled(A, B, RECT_N, rows, cols, ta, tb, cache=cache, err_rows=er, err_cols=ec,
                  label=f"rect {shape} {ta}{tb}")


# ---- the large stress workload ----

LARGE = 16384
BLOCK = [2, 100, 200, 254, 255]   # lines inside the cancellation block


@pytest.fixture(scope="module")
def large_inputs():
    held = {}

    def get(phi):
        if phi not in held:
            held.clear()
            s = phi_seed(5, phi)
            print(f"large phi={phi}: generating", flush=True)
            A = phi_matrix(LARGE, LARGE, phi, s)
            B = phi_matrix(LARGE, LARGE, phi, s + 1)
            A = cancellation_block(A, B, 256, 256, 1e-8, s + 2)
            held[phi] = (A, B, _samples(LARGE, LARGE, 500, ncols=128, cancel=True, extra=BLOCK),
                         {})
        return held[phi]

    yield get
    held.clear()


def test_large_accurate(large_inputs):
    # the paper's headline configuration: accurate mode, 12 hybrid moduli
    A, B, (rows, cols, er, ec), cache = large_inputs(1.0)
    check_sampled(A, B, 12, rows, cols, cache=cache, err_rows=er, err_cols=ec,
                  label="large phi=1")


LARGE_PHI6 = {"hybrid": 20, "int8": 24}


@pytest.mark.parametrize("moduli", ["hybrid", "int8"])
def test_large_wide_range_both_arms(large_inputs, moduli):
    # phi = 6: the FP8 hybrid path and the INT8 arm, each at the count that
    # reaches the same accuracy (1e-15)
    A, B, (rows, cols, er, ec), cache = large_inputs(6.0)
    check_sampled(A, B, LARGE_PHI6[moduli], rows, cols, moduli=moduli, cache=cache,
                  err_rows=er, err_cols=ec, label=f"large phi=6 {moduli}")
