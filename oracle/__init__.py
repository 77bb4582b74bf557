"""FP64 CPU oracle (test infrastructure only; see amm_oracle)."""
