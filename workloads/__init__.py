"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This package holds no part of the method's arithmetic: it only builds state
vectors (and request streams) of the shapes the paper and its benchmark
workloads use.  Both the CPU oracle and the GPU path consume its output;
neither is imported from here.
"""
from .states import (  # noqa: F401
    CONFIGS,
    CONFIG_FILE,
    BASE_SEED,
    SEED_N10,
    SEED_N16_BATCH,
    SEED_N20,
    SEED_SERVING,
    SEED_LARGE,
    WORKLOADS,
    haar,
    t_product,
    graph,
    graph_t,
    ising_couplings,
    ising_snapshot,
    computational_basis,
    plus_state,
    apply_random_clifford,
    to_dtype,
    workload_inputs,
    serving_requests,
    build_request,
    ising_energy,
    snapshot_couplings,
    random_adjacency,
    TFIM_PARAMS,
    product_angles,
    haar_u4,
    brickwork_pairs,
    brickwork_gates,
)
