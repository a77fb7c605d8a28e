"""MI355X-native graph-neural MPC hot path: GNN linearization and graph-sparse
condensing behind a C-ABI HIP library (``gnmpc``).

``workloads`` builds seeded synthetic inputs; ``gnmpc`` is the thin ctypes
binding over the C-ABI (it refuses to run without the built HIP library).
"""
