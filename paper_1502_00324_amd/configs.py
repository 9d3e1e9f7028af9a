"""Workload presets: the five encoder configurations (parameters only).

Each level is (B, L): range size B x B, domains 2B x 2B at step L.  S is the
contrast set num/den per level, the pool drops the lowest-entropy fraction
pct = (num, den) of the candidates, and a range splits when its RMS error
exceeds split_rms = (num, den) gray levels.
"""
from __future__ import annotations

from dataclasses import dataclass, field

from .synth import batch_shapes

K16 = tuple(range(17))  # S = {k/16 : k = 0..16}


@dataclass
class Workload:
    name: str
    images: list                      # (seed, width, height, n_rect)
    levels: list                      # (B, L) per quadtree level
    pct: tuple = (3, 10)              # drop the 30 % lowest-entropy candidates
    pool_max: int = 0
    s_num: tuple = K16
    s_den: int = 16
    split_rms: tuple = (8, 1)
    decode_iters: int = 0
    notes: str = ""
    extra: dict = field(default_factory=dict)


def _c4_images():
    seeds = list(range(1, 65))
    return [(s, w, h, 40) for s, (w, h) in zip(seeds, batch_shapes(seeds))]


WORKLOADS = {
    "c1_64": Workload("c1_64", [(0, 64, 64, 10)], [(8, 4), (4, 4)],
                      notes="64x64, B 8->4, L=4"),
    "c2_512": Workload("c2_512", [(0, 512, 512, 40)], [(16, 4), (8, 4), (4, 4)],
                       notes="512x512, B 16->8->4, L=4"),
    "c3_1024": Workload("c3_1024", [(0, 1024, 1024, 40)], [(8, 1), (4, 1)],
                        notes="1024x1024, B 8->4, L=1 (pool ~0.7M domains)"),
    "c4_batch64": Workload("c4_batch64", _c4_images(), [(16, 2), (8, 2), (4, 2)],
                           notes="64 images 128..1024, square or 2:1, B 16->8->4, L=2"),
    "c5_4096": Workload("c5_4096", [(0, 4096, 4096, 400)], [(32, 2), (16, 2), (8, 1), (4, 1)],
                        pct=(1, 2), decode_iters=8, notes="4096x4096, B 32->16->8->4, 50th percentile"),
    # the paper's own schedule: 4 steps 16->8->4->2, fixed pool size DN,
    # S = {0.1}, {0.2, 0.4}, {0.3, 0.8}, {0.5, 0.9}
    "paper_dn64": Workload("paper_dn64", [(0, 512, 512, 40)], [(16, 4), (8, 4), (4, 4), (2, 4)],
                           pct=(0, 1), pool_max=64,
                           s_num=((1,), (2, 4), (3, 8), (5, 9)), s_den=10, split_rms=(8, 1), decode_iters=8,
                           notes="paper schedule, DN = 64"),
}
