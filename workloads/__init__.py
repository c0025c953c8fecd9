"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package only *describes* inputs: gate lists (names, qubits, angles),
Pauli observables, parameter vectors and uniform streams, all drawn from
``numpy.random.Generator(PCG64(seed))``.  It holds none of the simulation
arithmetic (no gate matrices, no amplitudes) and imports neither the HIP
library nor the oracle.
"""
from .circuits import (Gate, layered_u3_cz, qft_circuit, qft_then_brick,
                       hardware_efficient_ansatz, random_pauli_sum,
                       random_planner_circuit, random_mixed_circuit,
                       ghz_circuit, w_circuit, uniform_stream, qubits_of,
                       config_circuit, rotation_cnot_circuit, mlp_init, SEEDS,
                       planner_mix_circuit, PLANNER_FAMILIES, noisy_layers)

__all__ = ["Gate", "layered_u3_cz", "qft_circuit", "qft_then_brick",
           "hardware_efficient_ansatz", "random_pauli_sum",
           "random_planner_circuit", "random_mixed_circuit", "ghz_circuit",
           "w_circuit", "uniform_stream", "qubits_of", "config_circuit",
           "rotation_cnot_circuit", "mlp_init", "SEEDS",
           "planner_mix_circuit", "PLANNER_FAMILIES", "noisy_layers"]
