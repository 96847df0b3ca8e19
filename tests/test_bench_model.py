"""The bench's algorithmic byte count per stage launch, checked on a
periodic straight mesh where every face is interior and every element
affine (no GPU)."""
import bench
import meshgen
from paper_1208_4772_amd import dg


def test_periodic_p5_bytes_per_element():
    r, s = dg.reference_nodes(5)
    case = meshgen.make_case("roofline", r, s, scale=0.01)
    b, info = bench.algorithmic_stage_bytes(case, 4)
    assert info == dict(curved=0, interior_sides=3 * case.K)
    # state in/out, R written every stage and read in 4 of 5: 4 Np (3 + 4/5)
    # floats; 3 faces x 6 nodes x 4 fields of neighbour traces; 13 floats of
    # geometry; 12 bytes of connectivity
    per_el = 4 * 21 * 4 * 3.8 + 3 * 6 * 4 * 4 + 13 * 4 + 12
    assert abs(b / case.K - per_el) < 1e-9
    assert abs(per_el - 1628.8) < 1e-9
    assert bench.stage_kernel_label(case, "fp32", 8) == "k_stage_mfma<5,false,8,false>"
    assert bench.stage_kernel_label(case, "fp64", 0) == "k_stage<double,5,false>"


def test_viscous_stage_counts_its_three_launches():
    r, s = dg.reference_nodes(3)
    case = meshgen.make_case("airfoil", r, s, scale=0.02, start="damped")
    assert case.av
    b_av, _ = bench.algorithmic_stage_bytes(case, 4)
    case.av = False
    b_inv, _ = bench.algorithmic_stage_bytes(case, 4)
    case.av = True
    # at least the gradient's output and the stage's read of it (8 Np
    # values each way) on top of the inviscid figure
    assert b_av - b_inv > case.K * 2 * 8 * case.Np * 4
    assert bench.stage_kernel_label(case, "fp32", 0) == \
        "k_sensor_elem<3> + k_avgrad<3> + k_stage_mfma<3,false,4,true>"
