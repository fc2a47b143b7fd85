"""The benchmark's byte accounting (host logic, no GPU): the method's bytes
per node-velocity and step, s (8 + 3 (d^2 + 1) / Q) (eight state accesses,
and the per-node metric and mass weight once per stage), and the per-launch
counts of the kernels."""
import bench


def _info(E, N, dim):
    n1 = N + 1
    np_ = n1 ** dim
    ni = (N - 1) ** dim
    return {"E": E, "np": np_, "dim": dim, "boundary_nodes_per_element": np_ - ni,
            "unique_nodes": E * ni + 1000, "groups": 1000}


def test_per_step_bytes():
    E, N, Q = 4096, 7, 27
    for s, per_nv in ((4, 36.44), (8, 72.89)):
        nv, step, _ = bench.algorithmic_bytes(_info(E, N, 3), Q, s)
        assert nv == E * 512 * Q
        assert abs(step / nv - s * (8 + 3 * 10 / Q)) < 1e-9
        assert abs(step / nv - per_nv) < 0.01


def test_per_launch_counts():
    E, N, Q, s = 64, 5, 19, 4
    info = _info(E, N, 3)
    _, _, per = bench.algorithmic_bytes(info, Q, s)
    np_, nb = info["np"], info["boundary_nodes_per_element"]
    G, ng = info["unique_nodes"], info["groups"]
    ni = np_ - nb
    assert per["stage23"] == s * (Q * G + 2 * Q * E * ni + Q * E * nb + E * np_ * 9 + 2 * E * ni)
    assert per["assembly"] == s * (Q * E * nb + 3 * Q * ng + 2 * ng) + 4 * (E * nb + ng)
    assert per["filter"] == s * 2 * Q * G


def test_stage_bytes_per_node_velocity():
    """One later SSPRK stage (element kernel and assembly together) reads the
    stage value and the post-collision state and writes the result (3 state
    accesses) plus the metric and mass weight: FP32 3D Q27 13.48 B, 2D Q9
    4 (3 + 5/9); the three stages add up to the step's figure."""
    b = bench.method_bytes(3, 27, 4)
    assert abs(b["later_stage"] - 4 * (3 + 10 / 27)) < 1e-12 and abs(b["later_stage"] - 13.48) < 0.005
    assert abs(b["stage1"] + 2 * b["later_stage"] - b["step"]) < 1e-12
    assert abs(bench.method_bytes(2, 9, 4)["later_stage"] - 4 * (3 + 5 / 9)) < 1e-12
