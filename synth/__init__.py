"""Seeded synthetic inputs shared by the GPU runtime's tests/benchmarks and the CPU oracle.

This package holds no part of any workload's arithmetic: it only draws inputs
(power-law graphs and their acyclic orientation, point sets, job traces).
"""
