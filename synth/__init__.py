"""Seeded synthetic inputs shared by the HIP path and the CPU oracle.

This package draws the random material of the scheme (secrets, key masks,
key errors, encryption masks and errors, messages, look-up tables) from a
seed.  It holds none of the scheme's arithmetic: both implementations take
these arrays as inputs and build keys, ciphertexts and test vectors from them
on their own.
"""
from .draws import (  # noqa: F401
    Q_DEFAULT,
    Q2_DEFAULT,
    CLASS_MIX,
    Params,
    PRESETS,
    discrete_gaussian,
    key_draws,
    enc_draws,
    messages,
    negacyclic_table,
    class_mix,
    poisson_arrivals,
)
