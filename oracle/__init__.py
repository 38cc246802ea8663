"""CPU FP64 oracle (test infrastructure only; see smpm_oracle's module docstring)."""
