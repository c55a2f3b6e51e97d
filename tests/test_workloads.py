"""The seeded input generators shared by tests, smoke check and benchmark:
reproducible, of the documented distributions, and the storage helpers
round-trip every storage order with leading-dimension padding."""
import numpy as np
import pytest

from workloads import (SEED_BASE, batch_shapes, cancellation_block, config_seed, from_colmajor,
                       integer_matrix, normal_matrix, phi_matrix, to_colmajor)


def test_config_seed_recipe():
    assert config_seed(0) == SEED_BASE == 2603_10634
    assert config_seed(2, 0) == SEED_BASE + 200
    assert config_seed(5, 1) == SEED_BASE + 510
    assert len({config_seed(c, q) for c in range(1, 6) for q in range(3)}) == 15


def test_phi_matrix_reproducible_and_distributed():
    a = phi_matrix(300, 200, 1.0, 7)
    assert a.dtype == np.float64 and a.shape == (300, 200)
    assert np.array_equal(a, phi_matrix(300, 200, 1.0, 7))
    assert not np.array_equal(a, phi_matrix(300, 200, 1.0, 8))
    # phi = 0: (U - 1/2) exactly, uniform on [-1/2, 1/2)
    u = phi_matrix(400, 500, 0.0, 9)
    assert u.min() >= -0.5 and u.max() < 0.5
    assert abs(u.mean()) < 0.01 and abs(u.var() - 1 / 12) < 0.002
    # the same draws scaled by exp(phi g): |x| / |u| = exp(phi g) has
    # log-standard-deviation phi
    for phi in (0.5, 2.0):
        x = phi_matrix(400, 500, phi, 9)
        ratio = np.log(np.abs(x[u != 0]) / np.abs(u[u != 0]))
        assert abs(ratio.std() - phi) < 0.02 * phi
        assert np.array_equal(np.sign(x), np.sign(u))


def test_normal_and_integer_matrices():
    g = normal_matrix(500, 400, 3)
    assert abs(g.mean()) < 0.01 and abs(g.std() - 1.0) < 0.01
    z = integer_matrix(300, 300, 5, 4)
    assert np.array_equal(z, np.rint(z)) and z.min() == -5 and z.max() == 5


def test_cancellation_block():
    A = phi_matrix(64, 96, 1.0, 11)
    B = phi_matrix(96, 48, 1.0, 12)
    C = cancellation_block(A, B, 16, 24, 1e-8, 13)
    assert np.array_equal(C[16:], A[16:])             # the other rows are untouched
    rel = np.abs(C[:16] @ B[:, :24]) / (np.abs(C[:16]) @ np.abs(B[:, :24]))
    assert rel.max() < 1e-7                           # products cancel to ~eps
    rel_out = np.abs(C[:16] @ B[:, 24:]) / (np.abs(C[:16]) @ np.abs(B[:, 24:]))
    assert np.median(rel_out) > 1e-3                  # outside the block they do not


@pytest.mark.parametrize("trans", ["N", "T", "C", "n", "t"])
@pytest.mark.parametrize("pad", [0, 3])
def test_colmajor_round_trip(trans, pad):
    op = phi_matrix(7, 5, 1.0, 14)
    r, c = op.shape
    stored_rows = r if trans in "Nn" else c
    buf, ld = to_colmajor(op, trans, ld=stored_rows + pad)
    assert ld == stored_rows + pad
    X = from_colmajor(buf, stored_rows, buf.size // ld, ld)
    back = X if trans in "Nn" else X.T
    assert np.array_equal(back, op)
    if pad:
        assert np.all(np.isnan(buf.reshape(-1, ld)[:, stored_rows:]))
    assert from_colmajor(buf, 0, 3, ld).shape == (0, 3)


def test_batch_shapes():
    s = batch_shapes(2000, 64, 4096, 15)
    assert s == batch_shapes(2000, 64, 4096, 15)
    x = np.array(s)
    assert x.min() >= 64 and x.max() <= 4096
    # log-uniform: the median of each dimension sits near sqrt(64 * 4096) = 512
    assert np.all(np.abs(np.log2(np.median(x, axis=0)) - 9) < 0.3)
