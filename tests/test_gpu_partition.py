"""Multi-partition BFS (Alg. 1) emulated on one GPU with the advance,
filter, package and combine kernels: global depths must equal the oracle's
BFS (and its serial BSP emulation O9)."""
import numpy as np
import pytest

import synth
from gpu_util import announce, gpu, need_gpu

pytestmark = gpu


@pytest.fixture(scope="module")
def part():
    need_gpu()
    from paper_1504_04804_amd import partition
    return partition


@pytest.mark.parametrize("nparts", [1, 2, 3, 4])
def test_partitioned_rmat(part, orc, nparts):
    off, col = synth.rmat_csr(12)
    owner = synth.owners(len(off) - 1, nparts)
    pb = part.PartitionedBFS(off, col, owner, nparts)
    for s in [0] + [int(x) for x in synth.sources(off, 3, seed=nparts)]:
        announce(f"partitioned bfs nparts={nparts} src={s}")
        got, it = pb.run(s)
        want, _, cnt, _ = orc.bfs(off, col, s)
        assert np.array_equal(got, want)
        assert np.array_equal(got, orc.bfs_partitioned(off, col, owner, nparts, s))
        assert it == len(cnt)


def test_partitioned_grid_and_medium(part, orc):
    off, col = synth.grid_csr(30, 41)
    owner = synth.owners(len(off) - 1, 4, seed=3)
    got, _ = part.PartitionedBFS(off, col, owner, 4).run(0)
    assert got.tolist() == [r + c for r in range(30) for c in range(41)]
    off, col = synth.rmat_csr(16)
    owner = synth.owners(len(off) - 1, 4)
    pb = part.PartitionedBFS(off, col, owner, 4)
    s = int(synth.sources(off, 1)[0])
    assert np.array_equal(pb.run(s)[0], orc.bfs(off, col, s)[0])
