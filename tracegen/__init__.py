"""Seeded synthetic trace generators (inputs for the checker and the oracle; no analysis code)."""
