"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only draws random numbers and shapes them into images and optical
fields; it contains none of the propagation or tensor-train arithmetic.  Every
generator takes an explicit ``seed`` (``numpy.random.default_rng``) and returns
float64 / complex128 host arrays; callers cast as they need.

The paper's own test photograph is not available, so these stand in for it:
natural images have a ~1/f amplitude spectrum (Sec. 2), and the optics
workloads of Sec. 5-6 are apertures carrying a phase field.
"""
from .fields import (  # noqa: F401
    blob_image, aperture_field, beam_grating_field, batch_specs,
    grating_beam_1d, smoothed_phase, random_field, gaussian_beam, beam_sum_1d,
)
