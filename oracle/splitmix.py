"""SplitMix64 (Steele, Lea, Flood, OOPSLA 2014), used to draw block split points.

Pinned by tests/test_oracle_maps.py against the generator's published first
outputs for seed 0 (tests/golden/splitmix64_seed0.txt).
"""
MASK = (1 << 64) - 1


class SplitMix64:
    def __init__(self, seed):
        self.s = seed & MASK

    def next(self):
        self.s = (self.s + 0x9E3779B97F4A7C15) & MASK
        z = self.s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
        return z ^ (z >> 31)
