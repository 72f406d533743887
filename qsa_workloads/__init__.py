"""Seeded synthetic workloads shared by the oracle tests and the benchmark.

This package holds workload descriptions and input generators only; it
contains none of the method's arithmetic.
"""
from .configs import (Species, Workload, slab_electron, slab_pair, cube256,
                      pair512, adjoint128, scan_instances, small_3d, CONFIGS)
from .generate import plasma_template, plasma_density, beam_species, beam, longitudinal_profile

__all__ = ["plasma_density", "Species", "Workload", "slab_electron", "slab_pair", "cube256",
           "pair512", "adjoint128", "scan_instances", "small_3d", "CONFIGS",
           "plasma_template", "beam_species", "beam", "longitudinal_profile"]
