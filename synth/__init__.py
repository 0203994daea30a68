"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

Holds no arithmetic of the optimiser itself: only scenario drawing."""
from .scenarios import (AC_FIELDS, N_AC_PAR, MIX_WEIGHTS, PRECISION, MOVES,  # noqa: F401
                        make_scenario, c1, c2, c3, c4, c5, paper_table, shrink)
