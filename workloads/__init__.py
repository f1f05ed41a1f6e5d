"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark:
meshes, partitions, materials and source currents.  Input arrays only; none
of the solver's arithmetic lives here."""
