"""Seeded synthetic inputs shared by the oracle and the GPU path.

``gen`` draws vectors; ``graph`` builds the fixed out-degree search graph.
Neither holds any arithmetic of the LeanVec search method.
"""
