"""The benchmark's algorithmic op count for k_propagate (the roofline's
numerator), pinned on the CPU for the benchmark workload: one 1024x436 pair,
k = 3, F and B1 with r = 8, B2 with r2 = 6, four sweeps and three random
searches per level.  The counts are derived by hand from the launch plan:
per field, level 8 runs sweep 1 alone, sweeps 2 and 3 as one pipelined pair
(the random search between them inside the launch), and sweep 4 paired with
the next level's sweep 1 (that level's entry inside the launch); the finest
level ends with sweep 4 alone -- 9 launches per field, 27 per pair, the count
the GPU bench measures."""
import bench


W, H, K = 1024, 436, 3
RADII = (8, 8, 6)


def test_grid_points_per_level():
    assert bench.grid_points(W, H, K) == [446464, 111616, 27904, 7040]


def test_sweep_ops_per_pair():
    pts = 446464 + 111616 + 27904 + 7040                      # 593,024 grid points, all levels
    # per sweep and point: 2 candidates x 2(2r+1) sliding-window terms x 2 ops
    want = sum(4 * pts * 2 * 2 * (2 * r + 1) * 2 for r in RADII)
    assert want == 891_908_096
    assert bench.propagate_ops_per_pair(W, H, K, RADII) == want


def test_per_point_stages_inside_launches():
    # one random search per level inside a sweep pair (all points of the
    # level) and three level entries inside cross-level pairs (the points of
    # levels 8, 4 and 2 carried to the finer grids)
    points = (7040 + 27904 + 111616 + 446464) + (7040 + 27904 + 111616)
    assert points == 739_584
    want = points * sum((2 * r + 1) ** 2 * 2 for r in RADII)
    assert want == 1_104_938_496
    assert bench.per_point_ops_in_sweep_launches(W, H, K, RADII) == want


def test_ops_per_launch_of_the_benchmark():
    total = bench.propagate_ops_per_pair(W, H, K, RADII) + bench.per_point_ops_in_sweep_launches(W, H, K, RADII)
    assert total == 1_996_846_592
    assert int(total / 27) == 73_957_281
