"""CPU oracle of the co-evolving-subspace step: TEST INFRASTRUCTURE ONLY.

Used by tests/, the smoke check and the benchmark's CPU-baseline leg; the
GPU library and its binding never import it.
"""
