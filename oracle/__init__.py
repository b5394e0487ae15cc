"""CPU oracle of the TLS search (test infrastructure only; see oracle.py)."""
