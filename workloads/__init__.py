"""Seeded synthetic inputs shared by the CPU oracle and the GPU library.

This package holds input data only: the element parameter set (a JSON file
written once by ``make_params.py``) and seeded geometry generators for the
workloads.  It contains none of the method's arithmetic (no integrals, no
Hamiltonian, no SCC), so both the oracle and the GPU path may import it.
"""

from .geometry import (  # noqa: F401
    ANGSTROM_TO_BOHR,
    System,
    water_cluster_cube,
    water_droplet,
    ion_pair_cluster,
    anthracene_crystal,
    pentacene_crystal,
    separated_water_pair,
    stream_droplet,
    load_params_json,
    params_path,
)
from .peptide import alanine_helix  # noqa: F401
