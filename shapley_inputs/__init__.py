"""Seeded synthetic inputs (games) shared by the oracle and the GPU path."""
from .games import (Game, Grid, grid_coords, isaacs_game, obstacle_game, dirichlet_1d_game,
                    two_stopper_game, two_stopper_exact, two_stopper_psi_bar, random_game,
                    scale_rows_to_stochastic)
from . import configs
