"""CPU oracle (test infrastructure only; see gqd_oracle's module docstring)."""
from .gqd_oracle import *  # noqa: F401,F403
from .gqd_oracle import (Model, SolverOpts, Stats, Counter, TRAP, MIDP, TRIPLE_JUMP, SUZUKI, OPTIMAL,
                         momentum_grid, model_from_item, apply_P, apply_F, apply_A, apply_H,
                         dense_H, inner, norm, energy, populations, symplectic_form, gmres,
                         givens, explicit_euler, implicit_euler, trapezoidal_step,
                         midpoint_step, composition_gammas, optimal_gammas, substep_fractions, propagate,
                         explicit_euler_propagate, implicit_euler_propagate, sod_start,
                         sod_propagate, diabatic_to_adiabatic, to_adiabatic, apply_H_diabatic,
                         exp_W, exp_T, split_operator_step, split_operator_propagate, adjoint,
                         population_loss)
