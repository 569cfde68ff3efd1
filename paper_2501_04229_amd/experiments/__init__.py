"""Experiment drivers that run the library on synthetic workloads (no oracle)."""
