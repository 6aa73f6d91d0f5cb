"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This package only draws random numbers and lays them out as arrays (phantoms,
coil maps, sampling masks and trajectories, k-space noise, initial weights).  It contains none
of the reconstruction arithmetic: no Fourier transform, no SENSE operator, no
solver and no network.  Both the FP64 oracle and the HIP path consume exactly
the arrays produced here (complex64 / float32), so a parity test measures
compute error only.
"""
from .generators import (  # noqa: F401
    phantom,
    coil_maps,
    pe_mask,
    kspace_noise,
    cnn_weights,
    vn_params,
    slice_inputs,
    batch_inputs,
    soft_slice_inputs,
    soft_batch_inputs,
    radial_trajectory,
    noncart_slice_inputs,
    noncart_batch_inputs,
    uneven_specs,
    uneven_inputs,
    UNEVEN_SHAPES,
    SEEDS,
)
