"""MI355X-native liquid-gas-solid lattice Boltzmann hot path (Bogner & Ruede)."""
