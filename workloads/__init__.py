"""Seeded, synthetic inputs shared by the oracle tests and the GPU path.

This package holds no arithmetic of the time stepper itself: it produces
meshes, coefficient fields sampled at node coordinates, initial states and
the pole/residue sets {alpha_m, b_m} that both sides receive as inputs.

Modules
-------
layout      node coordinates and the state layout the C-ABI expects
fields      wave-speed fields and initial states (pulses, eigenmodes, ...)
rational    least-squares residues b_m for poles on one vertical line
configs     the benchmark/parity workloads as plain recipes
"""
