"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package only draws random numbers and lays out op streams.  It holds
none of the emulation arithmetic: every gate or channel is emitted as
``(kind, qubits, params)`` with the physical parameters (angles, times,
probabilities) and each consumer builds its own matrices from them.
"""
from .circuits import (  # noqa: F401
    SEED_BASE,
    Op,
    c1_line_circuit,
    c2_grid_circuit,
    c3_all_to_all_circuit,
    c4_batch_instances,
    c5_ansatz_circuit,
    c5_draw_samples,
    c5_params,
    c5_structure,
    C5_N,
    C5_LAYERS,
    random_matrix_ops,
    count_gates,
    GATE_KINDS,
)
from .trajectories import TRAJ_SEED, damped_layer_circuit, random_tp_ops, traj_grid_circuit, uniforms  # noqa: F401,E402
