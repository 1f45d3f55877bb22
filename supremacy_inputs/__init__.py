"""Seeded synthetic inputs shared by the CPU oracle and the GPU library's tests.

This package only *generates inputs*: gate lists of Boixo-style random
supremacy circuits (gate names and qubit indices, never gate matrices),
seeded random state vectors and seeded Haar-random dense unitaries. It holds
none of the simulation arithmetic; the oracle and the GPU library each define
the named gates' matrices on their own.
"""
from .circuits import (  # noqa: F401
    Gate,
    Circuit,
    SplitMix64,
    supremacy_circuit,
    grid_edges,
    cz_pattern,
    batch_circuit_params,
    batch_circuit,
    blocked_circuit,
    with_haar_layers,
    mirror_circuit,
    drop_trailing_cz_layer,
    to_text,
    GATE_NAMES,
    DAGGER,
)
from .states import random_state, haar_unitary  # noqa: F401
