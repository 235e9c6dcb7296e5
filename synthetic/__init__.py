"""Seeded synthetic deblurring problems shared by the oracle tests, the GPU
tests and the benchmark.  Holds no solver arithmetic."""
from .problems import (Problem, true_image, psf_gaussian, psf_moffat_motion,
                       make_problem, small_gaussian, mid_anisotropic, large_moffat, large_moffat_periodic,
                       large_moffat_reflexive, large_moffat_motion_reflexive, psf_moffat,
                       batch_problem, lambda_grid, random_image, BATCH_SIZES, mixed_psf,
                       training_group, TRAIN_SEED0, VAL_SEED0, psf_defocus, study_problem,
                       STUDY_SEED0)

__all__ = ["Problem", "true_image", "psf_gaussian", "psf_moffat_motion",
           "make_problem", "small_gaussian", "mid_anisotropic", "large_moffat", "large_moffat_periodic",
           "large_moffat_reflexive", "large_moffat_motion_reflexive", "psf_moffat",
           "batch_problem", "lambda_grid", "random_image", "BATCH_SIZES", "mixed_psf",
           "training_group", "TRAIN_SEED0", "VAL_SEED0", "psf_defocus", "study_problem",
           "STUDY_SEED0"]
