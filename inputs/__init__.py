"""Seeded synthetic workloads shared by the tests, the smoke check and the benchmark."""
