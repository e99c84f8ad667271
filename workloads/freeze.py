"""Regenerate the frozen graph fixtures: ``python -m workloads.freeze``."""
from workloads import freeze_regular_graph

SIZES = [4, 6, 8, 10, 12, 14, 16, 18, 20, 60, 200, 210, 1000]

if __name__ == "__main__":
    for n in SIZES:
        for seed in (0, 1):
            print(freeze_regular_graph(n, 3, seed))
