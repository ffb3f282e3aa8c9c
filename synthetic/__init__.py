"""Seeded synthetic inputs (geometries, parameter draws) shared by the oracle and the library tests."""
