"""CPU reference oracle for the SSH hot path (Luo & Shrivastava, arXiv 1610.07328).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, float64 CPU
implementation of what the hot path computes, written from the paper.  It
exists so that the HIP path can be checked against it.  Only the tests, the
smoke check and the CPU-baseline leg of the benchmark may import or run it;
the product path never does.

It shares no code with the HIP path: neither imports the other.  Both take
their inputs from the seeded generators in ``paper_1610_07328_amd.datagen``,
which contain none of the method's arithmetic.

Every function is pinned by CPU tests against values and properties fixed by
the paper or by mathematics (worked examples, closed forms, brute force on
tiny inputs).  See ``tests/test_oracle_pins.py``.
"""
from .ssh_oracle import (  # noqa: F401
    EMPTY,
    KEY_EMPTY,
    HV_T_MAX,
    num_bits,
    num_shingles,
    sketch_series,
    sketch_batch,
    shingle,
    ln_table,
    cws,
    hv_encode,
    mix64,
    band_keys,
    wmh_int,
    wmh_int_batch,
    build_tables,
    probe,
    band_radius,
    dtw,
    rerank,
)
