"""FP64 CPU oracle (test infrastructure only; see avs_oracle's header)."""
