"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

Only input generation lives here (Hamiltonian integrals, bond allocation, random
canonical MPS, random vectors); none of the effective-Hamiltonian arithmetic does.
"""
