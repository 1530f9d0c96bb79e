"""FP64 CPU oracle (test infrastructure only; see tcflow_oracle)."""
