"""CPU oracle for the FP8 Ozaki-II DGEMM emulation.

Test infrastructure only: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.
"""
from .ozaki2_ref import (  # noqa: F401
    E4M3_MAX, E4M3_MIN_POS, E4M3_NONNEG, combine_alpha_beta, crt_reconstruct,
    cauchy_schwarz_norms, crt_weights, dgemm, digit_slices, digits_karatsuba, digits_square,
    e4m3_decode, e4m3_encode_exact, emulate, emulate_sampled, line_bounds, products, scaling,
    scaling_from_bounds, scaling_lines, exact_bound_product, hybrid_moduli,
    int8_moduli, inverse_scale, karatsuba_moduli, moduli_table, residue_product,
    residue_product_fp8, residues, round_up_e4m3, scale_exponent, smod,
    to_integers, ufp_exponents,
)
