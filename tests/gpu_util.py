"""Helpers shared by the GPU tests: moving seeded codes to the device and
comparing the library's output with the CPU oracle's."""
import numpy as np
import torch

import oracle


def to_dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int64)).cuda()


def as_u32(t: torch.Tensor) -> np.ndarray:
    return t.reshape(-1).cpu().numpy().view(np.uint32)


def assert_same(ids, dists, oids, odists, what=""):
    gi, gd = as_u32(ids), as_u32(dists)
    if not (np.array_equal(gi, oids) and np.array_equal(gd, odists)):
        bad = np.nonzero((gi != oids) | (gd != odists))[0]
        i = int(bad[0])
        raise AssertionError(f"{what}: {len(bad)} entries differ; first at {i}: "
                             f"gpu ({gi[i]}, {gd[i]}) oracle ({oids[i]}, {odists[i]})")


def oracle_knn(codes, queries, k):
    return oracle.knn(codes, queries, k)
