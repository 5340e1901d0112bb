"""Seeded synthetic inputs (design matrices and probit outcomes)."""
from .datasets import (Dataset, probit_design, sparse_beta, leading_beta, config1, config2,
                       config3, eq13, rare_event, batch_shapes, batch_dataset, bf16_bits, bf16_to_f32,
                       RARE_N, RARE_P, RARE_YBAR)

__all__ = ["Dataset", "probit_design", "sparse_beta", "leading_beta", "config1", "config2",
           "config3", "eq13", "rare_event", "batch_shapes", "batch_dataset", "bf16_bits", "bf16_to_f32",
           "RARE_N", "RARE_P", "RARE_YBAR"]
