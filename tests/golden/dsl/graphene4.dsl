# four-site graphene cell of Sec. 2.1 (matrices T_x, T_y, T_n), t = 1,
# written for the tests; per-orbital field v_{n,j} on the diagonal
dim 2
size 4
n_coeff_variable 4

nn -1 0
l0;
l1; 0|-1
l2;             3|-1
l3;

nn 1 0
l0; 1|-1
l1;
l2;
l3; 2|-1

nn 0 -1
l0; 3|-1
l1;
l2;
l3;

nn 0 1
l0;
l1;
l2;
l3; 0|-1

nn 0 0
l0; 0|v|0; 1|-1
l1; 0|-1;  1|v|1; 2|-1
l2; 1|-1;  2|v|2; 3|-1
l3; 2|-1;  3|v|3
