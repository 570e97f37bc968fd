// Batched persistent search (placeholder; the entry points live in kernels_search.hip for now).
