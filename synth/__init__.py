"""Seeded synthetic SUR workloads shared by the tests, the bench and the oracle.

This package only draws random inputs; it holds none of the estimation
method's arithmetic (no projections, no solves, no GLS formulas).
"""
from .sur import (  # noqa: F401
    SURInstance,
    SURBatch,
    config0,
    config1,
    config2,
    config2_sizes,
    config3,
    config4,
    small_batch,
    mc_sur,
    MVRInstance,
    var_regressors,
    mvrglm_var,
    e1_setup,
    e2_setup,
    tiny_integer_sur,
    CONFIGS,
)
