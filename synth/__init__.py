"""Seeded synthetic inputs shared by the GPU path, the oracle and the benchmarks.

This module only draws inputs: clean images, Poisson counts and filter banks.
It performs none of the denoiser's arithmetic (no Anscombe transform, no
filtering, no proximal step), so both sides of every parity check can use it
without sharing any of the method's code.

The paper evaluates on natural test images and a prior trained on BSDS300
patches (Section 2.6, Section 4); neither is available, so seeded synthetic
stand-ins with the same sizes and count levels are drawn here instead.
"""
from .images import clean_image, poisson_counts, noisy_pair
from .prior import dct_basis_no_dc, make_prior
from .workloads import (Job, load_params, oracle_config, fp32_config,
                        batch_config, serving_stream, lambda_for_peak,
                        data_term_for_peak, step_size_for)

__all__ = [
    "clean_image", "poisson_counts", "noisy_pair", "dct_basis_no_dc",
    "make_prior", "Job", "load_params", "oracle_config", "fp32_config",
    "batch_config", "serving_stream", "lambda_for_peak", "data_term_for_peak",
    "step_size_for",
]
