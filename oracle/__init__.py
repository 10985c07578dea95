"""FP64 CPU oracle (test infrastructure only; see cm_oracle.py)."""
