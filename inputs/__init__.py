"""Seeded inputs shared by the GPU path and the CPU oracle: alphabet, BLOSUM62,
background frequencies and synthetic workloads.  No alignment arithmetic."""
from .blosum import ALPHABET, N_RES, blosum62, background_frequencies, encode, decode  # noqa: F401
