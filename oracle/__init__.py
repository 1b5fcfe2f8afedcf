"""FP64 CPU oracle -- test infrastructure only (tests, smoke check, CPU baseline)."""
from .shapley_oracle import (OracleResult, transition_matrix, q_values, shapley_operator, greedy,
                             policy_system, evaluate_policies, policy_iteration, interp_value,
                             interp_policy, famg_pi, tied_states)
