"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle
checks.  Geometry, topology and parameter tables only."""
from .synth import (System, ZJ, MIX_GEOMETRIC, MIX_ARITHMETIC, MIX_SIXTHPOWER,
                    RELRES_CUTOFFS,  # noqa: F401
                    wrap, propane_liquid, neopentane_liquid, copolymer_melt,
                    random_molecules, two_atoms, perturbed_frames, WORKLOADS,
                    Batch, batch_of, mixed_liquid, replica_batch,
                    hexane_liquid, chain_positions)
