"""FP64 CPU oracle of the acoustic finite-difference path and of the CNN
gradient preconditioner (oracle.cnn).

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py, never by the product library.  It shares no
code with the GPU path.
"""
from . import wave
from . import cnn
from . import smooth
from . import resample
from .wave import (FD8, Grid, coefficients, laplacian, second_derivative, pad_edge,
                   fold_padding, sponge_profile, node_index, cfl_ratio,
                   laplacian_symbol_max, forward, misfit, gradient,
                   adjoint_source_transpose, energy, step)
from .revolve import binomial, forward_steps_closed_form, optimal_cost_table

__all__ = ["wave", "cnn", "smooth", "resample", "FD8", "Grid", "coefficients", "laplacian", "second_derivative",
           "pad_edge", "fold_padding", "sponge_profile", "node_index", "cfl_ratio",
           "laplacian_symbol_max", "forward", "misfit", "gradient",
           "adjoint_source_transpose", "energy", "step", "binomial",
           "forward_steps_closed_form", "optimal_cost_table"]
