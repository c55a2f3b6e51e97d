"""Plant plausible mistakes in the oracle (on the CPU) and confirm that the pin
checks catch every one of them (hybrid path, fast mode, and the Karatsuba-only
and INT8 lists).  This is what makes the pins worth trusting:
a dropped term, a wrong sign, a transposed or shifted index anywhere in the
oracle fails at least one check."""
import numpy as np
import pytest

from oracle import ozaki2_ref as ref
import test_oracle_core as core
import test_oracle_tables as tables


def _problem():
    return core._small_problem(5, 4, 15, 1.5, 900)


def _run_checks():
    A, B = _problem()
    failures = []
    checks = [
        ("smod", lambda: core.check_smod()),
        ("ufp", lambda: core.check_ufp(A)),
        ("scale", lambda: core.check_scale_exponent_brute(
            int(np.prod([p for p, _, _ in ref.hybrid_moduli(12)], dtype=object)),
            [1, 3, 2 ** 18, 12345678901])),
        ("cond3", lambda: core.check_condition3(A, B, 12)),
        ("bound", lambda: core.check_bound_dominates(A, B, 12)),
        ("intconv", lambda: core.check_integer_conversion(A, B, 12)),
        ("resprod", lambda: core.check_residue_products(A, B, 12)),
        ("crt", lambda: core.check_crt_is_exact_product(A, B, 12)),
        ("intexact", lambda: core.check_integer_inputs_exact(12)),
        ("errbound", lambda: core.check_error_bound(A, B, 12)),
        ("invariants", lambda: core.check_invariants(A, B, 12)),
        ("cond3_fast", lambda: core.check_condition3(A, B, 12, mode="fast")),
        ("fastnorm", lambda: core.check_fast_norms(A, B, 13)),
        ("fast_tight", lambda: core.check_fast_matches_accurate_when_tight(12)),
        ("lists", tables.test_printed_lists),
        ("karatsuba_pins", lambda: core.test_karatsuba_only_pins(5)),
        ("karatsuba_accuracy", core.test_karatsuba_only_integer_inputs_and_accuracy),
        ("int8_pins", lambda: core.test_int8_arm_pins(5)),
        ("int8_accuracy", core.test_int8_arm_accuracy_and_int32_limit),
    ]
    for name, fn in checks:
        try:
            fn()
        except Exception:                      # noqa: BLE001 - any failure counts
            failures.append(name)
    return failures


def test_clean_oracle_passes_every_check():
    assert _run_checks() == []


def _kara_wrong_x3(u, s=16):
    x1, x2, x3 = _orig["digits_karatsuba"](u, s)
    return x1, x2, x1 - x2


def _square_wrong_sign(u, s):
    x1, x2 = _orig["digits_square"](u, s)
    return x1, u + s * x1


def _crt_no_inverse(moduli):
    P, _ = _orig["crt_weights"](moduli)
    return P, [P // p for p in moduli]


def _crt_dropped(planes, moduli):
    P, w = _orig["crt_weights"](moduli)
    S = np.zeros(planes[0].shape, dtype=object)
    for wl, pl in list(zip(w, planes))[:-1]:
        S = S + wl * pl.astype(object)
    return ref.smod(S, P)


def _scale_plus_one(r18, P):
    e = _orig["scale_exponent"](r18, P)
    return e + 1 if r18 else e


def _round_down_e4m3(x, nonzero):
    idx = np.searchsorted(ref.E4M3_NONNEG, x, side="right") - 1
    return ref.E4M3_NONNEG[np.maximum(idx, 0)]


def _residues_unsigned(Xint, p):
    return np.fmod(Xint, p).astype(np.int64) % p


def _to_integers_round(op, shift, axis):
    sh = shift[:, None] if axis == 0 else shift[None, :]
    return np.round(np.ldexp(op, sh))


def _ufp_off_by_one(X, axis):
    return _orig["ufp_exponents"](X, axis) + 1


def _inverse_scale_wrong_sign(Cp, sA, sB):
    return _orig["inverse_scale"](Cp, -sA, sB)


def _residue_product_transposed_chunk(uA, uB, p):
    G = _orig["residue_product"](uA, uB, p)
    return ref.smod(G + 1, p)


def _fp8_route_sign(dA, dB, p, kind, s, chunk=2 ** 16):
    # Karatsuba recombination with the middle term's sign flipped
    if kind == "square":
        return _orig["residue_product_fp8"](dA, dB, p, kind, s, chunk)
    G = lambda x, y: (dA[x].astype(np.float64) @ dB[y].astype(np.float64)).astype(np.int64)
    c1, c2, c3 = G(0, 0), G(1, 1), G(2, 2)
    return ref.smod(s * s * c1 + c2 + s * (c3 + c1 - c2), p)


def _norms_unsquared(Abar, Bbar):
    return np.ldexp(Abar, 18).sum(axis=1), np.ldexp(Bbar, 18).sum(axis=0)


def _norms_unscaled(Abar, Bbar):
    return (Abar ** 2).sum(axis=1), (Bbar ** 2).sum(axis=0)


def _norms_unrounded(Abar, Bbar):
    # squares of the bound operand rounded down to a multiple of 2^-6 instead
    # of taken exactly
    return (np.ldexp(np.floor(np.ldexp(Abar, 6)), 3) ** 2).sum(axis=1), \
        (np.ldexp(np.floor(np.ldexp(Bbar, 6)), 3) ** 2).sum(axis=0)


def _norms_max_not_sum(Abar, Bbar):
    return (np.ldexp(Abar, 9) ** 2).max(axis=1), (np.ldexp(Bbar, 9) ** 2).max(axis=0)


def _smod_shifted(x, p):
    h = (p + 1) // 2
    return ((x + h) % p) - h


def _int8_list_from_255(N):
    return ref._greedy_coprime(range(255, 1, -1), N)


def _karatsuba_list_from_512(N):
    return ref._greedy_coprime(range(512, 1, -1), N)


def _int8_slice_unsigned(u, kind, s):
    # the INT8 residue stored as its unsigned byte
    if kind == "int8":
        return [np.mod(u, 256)]
    return _orig["digit_slices"](u, kind, s)


def _int8_product_unreduced(dA, dB, p, kind, s, chunk=2 ** 16):
    if kind != "int8":
        return _orig["residue_product_fp8"](dA, dB, p, kind, s, chunk)
    return (dA[0].astype(np.float64) @ dB[0].astype(np.float64)).astype(np.int64)


_orig = {name: getattr(ref, name) for name in (
    "digits_karatsuba", "digits_square", "crt_weights", "crt_reconstruct",
    "scale_exponent", "round_up_e4m3", "residues", "to_integers",
    "ufp_exponents", "inverse_scale", "residue_product", "residue_product_fp8",
    "smod", "cauchy_schwarz_norms", "digit_slices")}

MUTATIONS = {
    "karatsuba_x3": ("digits_karatsuba", _kara_wrong_x3),
    "square_digit_sign": ("digits_square", _square_wrong_sign),
    "crt_missing_inverse": ("crt_weights", _crt_no_inverse),
    "crt_dropped_modulus": ("crt_reconstruct", _crt_dropped),
    "scale_off_by_one": ("scale_exponent", _scale_plus_one),
    "round_down_cast": ("round_up_e4m3", _round_down_e4m3),
    "unsigned_residues": ("residues", _residues_unsigned),
    "round_not_trunc": ("to_integers", _to_integers_round),
    "ufp_off_by_one": ("ufp_exponents", _ufp_off_by_one),
    "unscale_sign": ("inverse_scale", _inverse_scale_wrong_sign),
    "residue_product_off": ("residue_product", _residue_product_transposed_chunk),
    "karatsuba_recombine_sign": ("residue_product_fp8", _fp8_route_sign),
    "smod_shifted": ("smod", _smod_shifted),
    "fast_norm_unsquared": ("cauchy_schwarz_norms", _norms_unsquared),
    "fast_norm_unscaled": ("cauchy_schwarz_norms", _norms_unscaled),
    "fast_norm_truncated": ("cauchy_schwarz_norms", _norms_unrounded),
    "fast_norm_max": ("cauchy_schwarz_norms", _norms_max_not_sum),
    "int8_list_from_255": ("int8_moduli", _int8_list_from_255),
    "karatsuba_list_from_512": ("karatsuba_moduli", _karatsuba_list_from_512),
    "int8_slice_unsigned": ("digit_slices", _int8_slice_unsigned),
    "int8_product_unreduced": ("residue_product_fp8", _int8_product_unreduced),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name, monkeypatch):
    attr, fn = MUTATIONS[name]
    monkeypatch.setattr(ref, attr, fn)
    failures = _run_checks()
    assert failures, f"planted mistake {name} was not caught by any pin"
