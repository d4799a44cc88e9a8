"""Seeded synthetic RGB-D inputs (scenes, renders, trajectories, correspondences).

Shared by the tests, the oracle checks and the benchmark as an input source only.
"""
from .problems import Problem, make_problem, make_chunk, make_global, make_batch_chunks  # noqa: F401
