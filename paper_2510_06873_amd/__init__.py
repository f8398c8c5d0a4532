"""MI355X-native per-step metadynamics bias pipeline (GPU-MetaD hot path).

The compute lives in ``libgpumetad.so`` (hand-written HIP for gfx950, C-ABI in
``include/gpumetad.h``); ``binding`` marshals torch tensors into it.
"""
from .binding import (Batch, ATOM_C, ATOM_CN, ATOM_NB, ATOM_Q6, CV_COORD, CV_COORD_Q6, CV_EXTERNAL, CV_Q6COUNT,
                      EXPORTS, FP32, FP64, GmError, Params, Pipeline, fes_reweight, fes_reweight_noalloc,
                      lattice_virial, lib, nearest_distance, nearest_distance_forces, torsion_forces, torsions,
                      version)

from . import autograd  # noqa: E402

__all__ = ["autograd", "Batch", "Pipeline", "Params", "GmError", "lib", "version", "EXPORTS", "CV_COORD", "CV_Q6COUNT",
           "CV_COORD_Q6", "CV_EXTERNAL", "FP32", "FP64", "ATOM_Q6", "ATOM_NB", "ATOM_C", "ATOM_CN", "torsions",
           "torsion_forces", "nearest_distance", "nearest_distance_forces", "lattice_virial", "fes_reweight",
           "fes_reweight_noalloc"]
