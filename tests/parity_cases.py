"""Case tables of the binary32 parity tests, shared by the GPU tests and by
the CPU test that shows their bars reject planted mistakes (tests/bars.py).
Inputs come from workloads' seeded generators with the seeds given here."""

# RKA with FP32 arithmetic: m, n, q, K, dtype, grid, allreduce, alpha
RKA32_CASES = [
    (600, 96, 8, 60, "f32", 0, 0, 1.0),      # one workgroup
    (700, 97, 4, 40, "f32", 0, 0, 0.9),      # scalar path
    (900, 4096, 8, 25, "f32", 0, 0, 1.0),    # many workgroups
    (900, 4096, 16, 20, "bf16", 0, 0, 1.3),
    (800, 2000, 11, 20, "f32", 16, 1, 1.0),  # all-gather exchange
    (800, 2000, 11, 20, "bf16", 16, 2, 0.8), # two-phase exchange
    (500, 3000, 40, 10, "f32", 0, 0, 1.5),   # 11-row bucket
]
RKA32_SEED_DATA, RKA32_SEED_SOLVE = 3, 5

# RKAB with FP32 arithmetic: m, n, q, bs, K, dtype, alpha
RKAB32_CASES = [
    (600, 96, 4, 5, 10, "f32", 1.0),
    (600, 97, 3, 4, 8, "bf16", 0.9),          # scalar path
    (400, 8192, 8, 6, 4, "bf16", 1.0),
    (300, 16000, 4, 5, 3, "f32", 0.7),        # iterate in LDS
    (500, 2048, 300, 2, 2, "f32", 1.2),       # more workers than workgroups
]
RKAB32_SEED_DATA, RKAB32_SEED_SOLVE = 4, 6

# batching form: shapes, (q, bs, tpr, K) and alpha per system; system s uses
# data seed BATCH_SEED0 + s and row-stream key BATCH_KEY + s
BATCH_SHAPES = [(300, 50), (1200, 97), (800, 200), (2000, 500), (5000, 1024), (700, 64),
                (900, 130), (3000, 2000), (640, 160), (1500, 256)]
BATCH_PARAMS = [(16, 4, 16, 6), (8, 8, 32, 5), (4, 16, 64, 4), (2, 20, 128, 3), (1, 30, 256, 3),
                (20, 2, 16, 5), (5, 3, 32, 7), (3, 10, 256, 2), (1, 1, 64, 40), (6, 6, 128, 4)]
BATCH_ALPHA = [1.0, 0.9, 1.0, 0.8, 1.0, 1.2, 1.0, 0.9, 1.0, 0.75]
BATCH_SEED0, BATCH_KEY = 100, 7

# one matrix shared by several right-hand sides: m, n, nrhs, q, bs, K, data seed, key
MULTI_RHS = (2000, 160, 7, 4, 8, 5, 31, 11)
