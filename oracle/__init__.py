"""CPU oracle for exact closeness centrality on homogeneous multilayer
networks.  Test infrastructure only: used by the tests, the smoke check and
the CPU-baseline leg of the benchmark, never by the product path."""
