"""MI355X (gfx950) solver for the Shapley equation of two-player zero-sum
stochastic games: policy iteration with an algebraic-multigrid inner solve
(AMGpi) and full multilevel policy iteration (FAMGpi), after Akian &
Detournay, arXiv:1107.1653.  The computation lives in libshapley.so (HIP);
this package only marshals arguments (see `shapley`)."""
from . import shapley  # noqa: F401
from .shapley import *  # noqa: F401,F403
