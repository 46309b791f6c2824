"""Seeded synthetic inputs (mechanisms, states, Newton data) shared by the
oracle-side tests and the GPU library's tests and benchmark. Holds none of the
kinetics arithmetic."""
from .mechgen import (WORKLOADS, Mechanism, Reaction, Species, config_mechanism,  # noqa: F401
                      make_mechanism, tiny_mechanism, ATM)
from .states import (NEWTON_GAMMA, conditioned_steps, config_states,  # noqa: F401
                     draw_newton_inputs, draw_states, pasr_fresh)
