"""Seeded synthetic inputs for the Li & Stephens all-vs-all copying model.

This package is shared by the CPU oracle and the GPU path. It generates
haplotype matrices, recombination probabilities and target lists, and packs
haplotypes into the bit layout both sides read. It holds none of the model's
arithmetic: no emissions, transitions, recursions or posteriors.
"""

from .mosaic import (
    MosaicSpec,
    mosaic_haplotypes,
    rho_from_spacings,
    spacings,
    evenly_spaced_targets,
    seeded_recipients,
)
from .packing import pack_haplotypes, unpack_haplotypes, packed_stride_words, packed_bytes
from .configs import CONFIGS, get_config, make_inputs

__all__ = [
    "MosaicSpec",
    "mosaic_haplotypes",
    "rho_from_spacings",
    "spacings",
    "evenly_spaced_targets",
    "seeded_recipients",
    "pack_haplotypes",
    "unpack_haplotypes",
    "packed_stride_words",
    "packed_bytes",
    "CONFIGS",
    "get_config",
    "make_inputs",
]
