"""Batched Montgomery-type modular arithmetic on MI355X (gfx950).

Operations (all in HIP kernels of libmont.so, called through its C ABI):

* ``setup(N, w)``                 per-modulus constants (Section 1 of the paper)
* ``redc / mul``                  classic REDC, signed Montgomery (Algorithm 1),
                                  Plantard (Algorithm 2), signed Plantard
                                  (Algorithm 3), Huang's variant with alpha >= 1
                                  (Algorithm 4), at 16/32/64-bit words
* ``mul_const``                   the product by one fixed operand (precomputed b N^{-1})
* ``mul_rns``                     the product over residue-number-system rows
* ``crt``                         integers from residue rows (multi-modulus CRT)
* ``ntt``                         batched number-theoretic transforms (Montgomery or Plantard twiddles)
* ``pow``                         x^e mod N through the Montgomery representation
* ``redc_range``                  REDC over a generated range of T
* ``Batch``                       ragged batches in one persistent launch
* ``serve``                       the continuous-batching request loop
* ``library``, ``debug_violations``  the MONT_DEBUG build and its precondition counter
"""
from ._lib import (  # noqa: F401
    BATCH_DYNAMIC, BATCH_GRAPH, BATCH_NONTEMPORAL, BATCH_TUNE, CLASSIC, E_BUSY, E_CANCELED, E_DEVICE, E_INVAL, OP_MUL, OP_POW, OP_REDC, PLANTARD, SIGNED,
    SIGNED_PLANTARD, SIGNED_PLANTARD_ALPHA, VARIANTS, Batch, Ctx, MontError, batch_run_noalloc, elem_dtype, get_launch,
    Server, crt, debug_violations, header_functions, library, load, mul, mul_const, mul_rns, ntt, pools, pow,
    redc, redc_range, set_launch, setup, stream_ref, tune_mul, valu_ref, version,
)
