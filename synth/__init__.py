"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package holds no arithmetic of the method: it only names the workloads
(leg sector lists, precisions, seeds) and draws the Gaussian numbers that fill
tensor blocks.  How those numbers are laid out into blocks (canonical block
order, row-major within a block) is decided independently by each consumer.
"""
from .configs import CONFIGS, config, batched_draws, binomial_sectors, virtual_sectors_for_D
from .draw import draw, TENSOR_INDEX, SITE_AND_ENV

__all__ = ["CONFIGS", "config", "batched_draws", "binomial_sectors",
           "virtual_sectors_for_D", "draw", "TENSOR_INDEX", "SITE_AND_ENV"]
