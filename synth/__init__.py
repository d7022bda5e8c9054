"""Seeded synthetic hypergraph generators (inputs only; no matching logic).

Both the GPU path's tests and the oracle read their inputs from here.  The
module draws random hypergraphs of the shapes the paper evaluates on (sizes,
degree skew, hub vertices, weight ranges) and lays them out in the dual
compressed form; it performs none of the matching arithmetic.
"""
from .gen import (Batch, Hypergraph, batch_from_instances, config_batched, config_delaunay,
                  config_hub_stress, config_plain, config_power_law, config_rgg,
                  config_served_pool, from_edge_lists, from_pairs, random_instance, rgg_pairs,
                  shuffle_batch, shuffle_lists, transpose)

__all__ = ["Batch", "Hypergraph", "batch_from_instances", "config_batched", "config_delaunay",
           "config_hub_stress", "config_plain", "config_power_law", "config_rgg",
           "config_served_pool", "from_edge_lists", "from_pairs", "random_instance", "rgg_pairs",
           "shuffle_batch", "shuffle_lists", "transpose"]
