"""FP64 CPU oracle of the APSM detector.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the library or its Python binding.
"""
from .apsm_oracle import *  # noqa: F401,F403
from .apsm_oracle import (APSMParams, Filter, Trainer, TermListTrainer,  # noqa: F401
                          train, train_from_pilots, detect, detect_planar,
                          evaluate_many, decide, symbol_errors, training_sequence,
                          real_split, kappa_gauss, kappa_lin, kappa_sum, gram,
                          boundary_distance, axis_thresholds, window, beta)
