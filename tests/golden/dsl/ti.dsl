# 3D topological insulator (Sec. 2.2), t = 1, m = 2, written for the tests
# from the hopping -(t/2)(G1 - i G_{j+1}) with G1 = tau_z sigma_0,
# G_{j+1} = tau_x sigma_j, orbital o = 2 tau + sigma.
# Block at offset d: y[s][row] += value * x[s + d][col]; d = -e_j carries the
# hop itself, d = +e_j its adjoint.
dim 3
size 4
n_coeff_const 1
n_coeff_variable 1
coeff_const_default 2

nn -1 0 0
l0; 0|-0.5; 3|0.5i
l1; 1|-0.5; 2|0.5i
l2; 2|0.5;  1|0.5i
l3; 3|0.5;  0|0.5i

nn 1 0 0
l0; 0|-0.5; 3|-0.5i
l1; 1|-0.5; 2|-0.5i
l2; 2|0.5;  1|-0.5i
l3; 3|0.5;  0|-0.5i

nn 0 -1 0
l0; 0|-0.5; 3|0.5
l1; 1|-0.5; 2|-0.5
l2; 2|0.5;  1|0.5
l3; 3|0.5;  0|-0.5

nn 0 1 0
l0; 0|-0.5; 3|-0.5
l1; 1|-0.5; 2|0.5
l2; 2|0.5;  1|-0.5
l3; 3|0.5;  0|0.5

nn 0 0 -1
l0; 0|-0.5; 2|0.5i
l1; 1|-0.5; 3|-0.5i
l2; 2|0.5;  0|0.5i
l3; 3|0.5;  1|-0.5i

nn 0 0 1
l0; 0|-0.5; 2|-0.5i
l1; 1|-0.5; 3|0.5i
l2; 2|0.5;  0|-0.5i
l3; 3|0.5;  1|0.5i

# on-site: m G1 (constant c0 = m) plus the disorder V_n on every orbital
nn 0 0 0
l0; 0|c|0;  0|v|0
l1; 1|c|0;  1|v|0
l2; 2|-2;   2|v|0
l3; 3|-2;   3|v|0
