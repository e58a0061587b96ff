"""MI355X exhaustive dense-QUBO solver (prefix-suffix decomposition + Gray-code walk)."""
