"""CPU FP64 oracle (test infrastructure only; see slepian_oracle's header)."""
