"""The benchmark's byte accounting (host logic, no GPU): the method's bytes
per node-velocity and step, s (8 + 3 (m + 1) / Q) with m the metric values
per node (dim^2 on curved elements, dim^2 / np on affine ones), and the
per-launch counts of the dominant kernels."""
import bench


def _info(E, N, dim, ea):
    n1 = N + 1
    np_ = n1 ** dim
    ni = (N - 1) ** dim
    return {"E": E, "np": np_, "dim": dim, "boundary_nodes_per_element": np_ - ni,
            "unique_nodes": E * ni + 1000, "groups": 1000, "affine_elements": ea}


def test_per_step_bytes_curved_and_affine():
    E, N, Q = 4096, 7, 27
    for s, curved, affine in ((4, 36.44, 32.45), (8, 72.89, 64.90)):
        nv, step, _ = bench.algorithmic_bytes(_info(E, N, 3, 0), Q, s)
        assert abs(step / nv - curved) < 0.01
        nv, step, _ = bench.algorithmic_bytes(_info(E, N, 3, E), Q, s)
        # metric d^2 per element instead of per node: d^2 / np per node
        exact = s * (8 + 3 * (1 + 9 / 512) / Q)
        assert abs(step / nv - exact) < 1e-9 and abs(step / nv - affine) < 0.01


def test_per_launch_metric_term():
    E, N, Q, s = 64, 5, 19, 4
    _, _, cur = bench.algorithmic_bytes(_info(E, N, 3, 0), Q, s)
    _, _, aff = bench.algorithmic_bytes(_info(E, N, 3, E), Q, s)
    np_ = (N + 1) ** 3
    for k in ("stage1", "stage23"):
        assert cur[k] - aff[k] == s * (E * np_ * 9 - E * 9)
    # the assembly, filter and closure kernels do not depend on it
    for k in ("assembly", "filter", "features", "network"):
        assert cur[k] == aff[k]
