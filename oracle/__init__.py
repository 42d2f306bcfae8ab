"""CPU FP64 oracle (test infrastructure only; see ``bta_oracle``)."""
from .bta_oracle import (pobtaf, pobtasi, pobtas, logdet, grad_logdet_quad, dense,
                         dense_lower_factor, pattern, rel_block_errors)

__all__ = ["pobtaf", "pobtasi", "pobtas", "logdet", "grad_logdet_quad", "dense",
           "dense_lower_factor", "pattern", "rel_block_errors"]
