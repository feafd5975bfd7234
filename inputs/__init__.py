"""Seeded inputs shared by the GPU path and the CPU oracle: alphabet, BLOSUM62,
background frequencies and synthetic workloads.  No alignment arithmetic."""
from .blosum import (ALPHABET, ALPHABET24, N_RES, blosum62, blosum62_24, background_frequencies,  # noqa: F401
                     encode, decode)
