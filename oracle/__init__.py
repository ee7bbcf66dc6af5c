"""FP64 CPU oracle (test infrastructure only; see ek_oracle.c)."""
